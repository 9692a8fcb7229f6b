"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and rejects invalid configurations before touching a GPU."""
import ctypes

import pytest

import paper_2510_08782_amd as gan


def test_library_exports_every_header_symbol():
    lib = gan.lib()
    syms = gan.header_symbols()
    assert len(syms) == 27
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
    assert ctypes.sizeof(gan.StepInfo) == 592


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


def test_host_least_squares_matches_the_oracle():
    """The library's host solve of the NGMRES least-squares problem (Cholesky,
    else the pseudo-inverse) against the oracle's, from the same Gram matrix:
    a full-rank window (Cholesky), and windows with a repeated column and with
    more columns than entries (pseudo-inverse, the minimum-norm solution,
    also checked against numpy's lstsq on the explicit difference matrix)."""
    import numpy as np

    from oracle import ngmres as ong
    rng = np.random.default_rng(5)
    r = rng.standard_normal(40)
    full = [rng.standard_normal(40) for _ in range(5)]
    dup = full[:3] + [full[1].copy()] + full[3:]
    wide = [rng.standard_normal(6) for _ in range(9)]
    r6 = rng.standard_normal(6)
    for rr, gs, want_fb in ((r, full, False), (r, dup, True), (r6, wide, True)):
        G = ong.gram([rr] + gs)
        beta, fb = gan.lsq(G)
        assert fb == want_fb
        np.testing.assert_allclose(beta, ong.lsq_from_gram(G), rtol=1e-9, atol=1e-11)
        if want_fb:
            np.testing.assert_allclose(beta, ong.lsq_direct(rr, gs), rtol=1e-7, atol=1e-9)
    bad = np.eye(3)
    bad[0, 1] = 1.0           # not symmetric
    with pytest.raises(gan.GanmresError):
        gan.lsq(bad)
