"""The C-ABI library loads and exports every entry point include/boltz.h
declares; argument validation that precedes any HIP call (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "boltz.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(boltz_[a-z_0-9]+)\s*\(", text)))


def _lib():
    from paper_1005_5405_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libboltz.so is not built (run __graft_entry__.build())")
    return binding.load_library(), binding


def test_header_declares_the_hot_path():
    names = _declared()
    for fn in ("boltz_stream", "boltz_collide", "boltz_moments", "boltz_step", "boltz_step_adjoint",
               "boltz_stream_adjoint", "boltz_collide_adjoint", "boltz_lid_shear_adjoint", "boltz_create",
               "boltz_destroy"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    L, binding = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(binding.EXPORTS) == set(_declared())


def test_null_and_invalid_arguments_are_rejected_before_any_device_call():
    L, binding = _lib()
    ctx = ctypes.c_void_p()
    assert L.boltz_create(None, ctypes.byref(ctx)) == binding.EINVAL
    assert "null" in L.boltz_last_error(None).decode()
    bad = [dict(nx=1), dict(nv=(0, 4, 4)), dict(nv=(256, 4, 4)), dict(eps=0.0), dict(order=3),
           dict(n_pairs=2**31), dict(dt=1.0), dict(vmax=(0.0, 1.0, 1.0)), dict(sample_group=-1),
           dict(mix16=17), dict(flags=16),
           # the sequential update needs shared samples and has no adjoint
           dict(flags=8, sample_group=1), dict(flags=8 | 2, sample_group=0),
           # stretched spatial cells: 0 < r < 1, first-order streaming, no adjoint
           dict(rx=0.9, order=2), dict(ry=1.5, order=1), dict(rx=-0.1, order=1), dict(rx=0.9, order=1, flags=2),
           # the 12-bit Maxwellian law alone cannot draw the outer nodes of 8 cells on [-4, 4]
           dict(mix16=0, vmax=(4.0, 4.0, 4.0)), dict(mix16=0, nv=(20, 20, 20), vmax=(5.0, 5.0, 5.0)),
           # stretched velocity cells need 0 < rv < 1 and even counts
           dict(rv=1.5), dict(rv=-0.2), dict(rv=0.9, nv=(8, 7, 8))]
    base = dict(nx=8, ny=8, nv=(8, 8, 8), vmax=(3.0, 3.0, 3.0), delta=1.0, eps=0.1, cfl=0.5, dt=0.0, order=2,
                bc=0, n_pairs=100, sample_group=1, seed=1, cavity_id=0, flags=0, mix16=4, rv=0.0)
    for over in bad:
        kw = dict(base, **over)
        p = binding._Problem(kw["nx"], kw["ny"], (ctypes.c_int32 * 3)(*kw["nv"]),
                             (ctypes.c_double * 3)(*kw["vmax"]), kw["delta"], kw["eps"], kw["cfl"], kw["dt"],
                             kw["order"], kw["bc"], kw["n_pairs"], kw["sample_group"], kw["seed"],
                             kw["cavity_id"], kw["flags"], kw["mix16"], kw["rv"], kw.get("rx", 0.0),
                             kw.get("ry", 0.0))
        rc = L.boltz_create(ctypes.byref(p), ctypes.byref(ctx))
        assert rc == binding.EINVAL, (over, rc)
        if over.get("mix16") == 0:
            assert "mix16 = 0" in L.boltz_last_error(None).decode()
    # a velocity grid whose per-cell tiles exceed the 160 KB LDS
    kw = dict(base, nv=(30, 30, 30))
    p = binding._Problem(kw["nx"], kw["ny"], (ctypes.c_int32 * 3)(*kw["nv"]), (ctypes.c_double * 3)(*kw["vmax"]),
                         kw["delta"], kw["eps"], kw["cfl"], kw["dt"], kw["order"], kw["bc"], kw["n_pairs"],
                         kw["sample_group"], kw["seed"], kw["cavity_id"], kw["flags"], kw["mix16"])
    assert L.boltz_create(ctypes.byref(p), ctypes.byref(ctx)) == binding.EUNSUPPORTED
    # calls on a null context
    assert L.boltz_stream(None, None, None, None, None) == binding.EINVAL
    assert L.boltz_collide(None, None, None, 0, 0, None, None) == binding.EINVAL
    assert L.boltz_moments(None, None, None, None, None, None) == binding.EINVAL
    assert L.boltz_step(None, None, None, None, 0, None) == binding.EINVAL
    assert L.boltz_step_adjoint(None, None, None, None, None, None, 0, None) == binding.EINVAL
    assert L.boltz_stream_adjoint(None, None, None, None, None, None, None) == binding.EINVAL
    assert L.boltz_collide_adjoint(None, None, None, None, 0, 0, None) == binding.EINVAL
    assert L.boltz_lid_shear_adjoint(None, None, None, 1.0, None, None, None) == binding.EINVAL


def test_batch_arguments_are_rejected_before_any_device_call():
    L, binding = _lib()
    b = ctypes.c_void_p()
    p = binding._problem(nx=8, ny=8, nv=8, vmax=3.0, delta=1.0, eps=0.1, n_pairs=10)
    q = binding._problem(nx=8, ny=8, nv=8, vmax=3.0, delta=1.0, eps=0.1, n_pairs=10, order=1)
    r = binding._problem(nx=8, ny=8, nv=(8, 8, 6), vmax=3.0, delta=1.0, eps=0.1, n_pairs=10)
    assert L.boltz_batch_create(None, 1, ctypes.byref(b)) == binding.EINVAL
    assert L.boltz_batch_create((binding._Problem * 1)(p), 0, ctypes.byref(b)) == binding.EINVAL
    assert L.boltz_batch_create((binding._Problem * 2)(p, q), 2, ctypes.byref(b)) == binding.EINVAL
    assert "order" in L.boltz_batch_last_error(None).decode()
    assert L.boltz_batch_create((binding._Problem * 2)(p, r), 2, ctypes.byref(b)) == binding.EINVAL
    assert "nv[2]" in L.boltz_batch_last_error(None).decode()
    s = binding._problem(nx=8, ny=8, nv=8, vmax=3.0, delta=1.0, eps=0.1, n_pairs=10, sample_group=0, flags=8)
    assert L.boltz_batch_create((binding._Problem * 2)(p, s), 2, ctypes.byref(b)) == binding.EINVAL
    assert "Jacobi" in L.boltz_batch_last_error(None).decode()
    q1 = binding._problem(nx=8, ny=8, nv=8, vmax=3.0, delta=1.0, eps=0.1, n_pairs=10, order=1)
    t1 = binding._problem(nx=8, ny=8, nv=8, vmax=3.0, delta=1.0, eps=0.1, n_pairs=10, order=1, rx=0.9, ry=0.9)
    assert L.boltz_batch_create((binding._Problem * 2)(q1, t1), 2, ctypes.byref(b)) == binding.EINVAL
    assert "uniform spatial" in L.boltz_batch_last_error(None).decode()
    assert L.boltz_batch_step(None, None, None, None, None) == binding.EINVAL
    assert L.boltz_batch_query(None, None) == binding.EINVAL
    assert L.boltz_batch_problem(None, 0) is None
