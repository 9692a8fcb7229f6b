"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and rejects invalid configurations before touching a GPU."""
import ctypes

import pytest

import paper_2510_08782_amd as gan


def test_library_exports_every_header_symbol():
    lib = gan.lib()
    syms = gan.header_symbols()
    assert len(syms) == 22
    for name in syms:
        assert hasattr(lib, name), name
    for name in ["ganmres_eval_objective", "ganmres_eval_gradient", "ganmres_apply_precond",
                 "ganmres_step", "ganmres_create_batch"]:
        assert name in syms


def test_kernel_names_and_struct_layout():
    lib = gan.lib()
    n = lib.ganmres_kernel_count()
    names = [lib.ganmres_kernel_name(i).decode() for i in range(n)]
    assert "sl_step" in names and "deriv_axis" in names
    assert lib.ganmres_kernel_name(n) == b""
    # ctypes mirrors of the C structs: sizes as gcc lays them out on x86-64
    assert ctypes.sizeof(gan.Config) == 48
    assert ctypes.sizeof(gan.SolverParams) == 72
    assert ctypes.sizeof(gan.StepInfo) == 584


@pytest.mark.parametrize("bad", [
    dict(dim=4), dict(n=(7, 64, 1)), dict(n=(2048, 64, 1)), dict(nt=0), dict(alpha=0.0),
    dict(reg_order=4), dict(model=5), dict(dtype=3), dict(checkpoint_every=0),
    dict(model=gan.CONTINUITY, incompressible=1),
])
def test_create_rejects_invalid_config_without_device_work(bad):
    base = dict(dim=2, n=(64, 64, 1), nt=4, model=gan.ADVECTION, incompressible=0,
                reg_order=1, alpha=1e-2, dtype=gan.F64, checkpoint_every=1)
    base.update(bad)
    cfg = gan.Config(base["dim"], (ctypes.c_int * 3)(*base["n"]), base["nt"], base["model"],
                     base["incompressible"], base["reg_order"], base["alpha"], base["dtype"],
                     base["checkpoint_every"])
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)      # never dereferenced: validation fails first
    rc = gan.lib().ganmres_create(ctypes.byref(cfg), dummy, dummy, None, ctypes.byref(h))
    assert rc == -1
    assert gan.lib().ganmres_last_error(None)
    assert not h.value


@pytest.mark.parametrize("count,dim,alpha", [
    (0, 2, None), (65, 2, None), (2, 3, None), (2, 2, (1e-2, 0.0)), (2, 2, (1e-2, -1.0)),
])
def test_create_batch_rejects_invalid_batches(count, dim, alpha):
    n = (32, 32, 32) if dim == 3 else (32, 32, 1)
    cfg = gan.Config(dim, (ctypes.c_int * 3)(*n), 4, gan.ADVECTION, 0, 1, 1e-2, gan.F64, 1)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)      # never dereferenced: validation fails first
    al = (ctypes.c_double * len(alpha))(*alpha) if alpha else None
    rc = gan.lib().ganmres_create_batch(ctypes.byref(cfg), count, al, dummy, dummy, None,
                                        ctypes.byref(h))
    assert rc == -1
    assert gan.lib().ganmres_last_error(None)
    assert not h.value


def test_null_arguments_are_rejected():
    lib = gan.lib()
    assert lib.ganmres_eval_objective(None, None, 0, None, None) == -1
    assert lib.ganmres_step(None, None, None, None) == -1
    assert lib.ganmres_destroy(None) == 0
    assert lib.ganmres_batch_count(None) == 0
    assert lib.ganmres_batch_values(None, None, None) == -1
