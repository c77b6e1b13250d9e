"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/gamblet.h, and validates arguments on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "gamblet.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(gbl_\w+)\s*\(", src, flags=re.M)))


def _lib():
    import paper_1503_03467_amd as P
    return P, P.lib()


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 8
    _, L = _lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_version_and_defaults():
    P, L = _lib()
    assert L.gbl_version() == 10000
    o = P.make_opts()
    assert o.rho == 3 and o.precision == 1 and o.rtol == 1e-8


@pytest.mark.parametrize("q", [1, 13, -2])
def test_bad_q_rejected(q):
    P, _ = _lib()
    with pytest.raises(P.GambletError) as e:
        P.workspace_bytes(q, P.make_opts())
    assert e.value.code == -1


@pytest.mark.parametrize("field,value", [("rho", 0), ("rho", 5), ("precision", 7), ("rtol", 0.0),
                                         ("rtol", 2.0), ("max_outer", 0), ("max_rhs", 0), ("inner_kind", 3),
                                         ("window_tol", -1.0), ("window_tol", 1000.0),
                                         ("kappa", 1.0), ("kappa_coarse", 0.5), ("inner_iters", 33),
                                         ("inner_iters_coarse", 33)])
def test_bad_options_rejected(field, value):
    P, _ = _lib()
    o = P.make_opts()
    setattr(o, field, value)
    with pytest.raises(P.GambletError):
        P.workspace_bytes(6, o)


def test_workspace_grows_with_q_and_precision():
    P, _ = _lib()
    sizes = [P.workspace_bytes(q, P.make_opts(precision="mixed")) for q in range(2, 11)]
    assert all(b > a for a, b in zip(sizes, sizes[1:]))
    assert P.workspace_bytes(9, P.make_opts(precision="fp64")) > P.workspace_bytes(9, P.make_opts())


def test_null_arguments_rejected():
    P, L = _lib()
    o = P.make_opts()
    ctx = ctypes.c_void_p()
    assert L.gbl_build(ctypes.byref(ctx), 6, None, ctypes.byref(o), ctypes.c_void_p(16), 1 << 30, None) == -1
    assert b"a_dev" in L.gbl_last_error(None)
    assert L.gbl_build(ctypes.byref(ctx), 6, ctypes.c_void_p(16), ctypes.byref(o), None, 1 << 30, None) == -1
    assert L.gbl_build(None, 6, ctypes.c_void_p(16), ctypes.byref(o), ctypes.c_void_p(16), 1 << 30, None) == -1
    assert L.gbl_solve(None, 1, None, None, None, None) == -1
    assert L.gbl_destroy(None) == 0
    flags = ctypes.c_uint(7)
    assert L.gbl_build_flags(None, ctypes.byref(flags)) == -1
    # batched calls validate their arrays before touching the device
    assert L.gbl_build_batched(0, None, None, None, None, None, None, None, None) == -1
    assert b"batched build" in L.gbl_last_error(None)
    assert L.gbl_solve_batched(0, None, None, None, None, None, None, None) == -1
    assert b"batched solve" in L.gbl_last_error(None)


def test_short_workspace_rejected_before_any_device_work():
    P, L = _lib()
    o = P.make_opts()
    need = P.workspace_bytes(6, o)
    ctx = ctypes.c_void_p()
    rc = L.gbl_build(ctypes.byref(ctx), 6, ctypes.c_void_p(16), ctypes.byref(o), ctypes.c_void_p(16),
                     need - 1, None)
    assert rc == -4
    assert b"workspace" in L.gbl_last_error(None)


def test_default_options():
    P, _ = _lib()
    o = P.make_opts()
    assert (o.rho, o.precision, o.max_outer, o.inner_kind) == (3, 1, 100, 0)
    assert (o.inner_iters, o.inner_iters_coarse, o.kappa, o.kappa_coarse) == (16, 2, 200.0, 10.0)
    cg = P.make_opts(inner="cg", inner_iters=40)
    assert cg.inner_kind == 1 and P.workspace_bytes(6, cg) > 0   # CG budgets are not capped at 32


def test_level_q_calls_validate_arguments():
    """The level-q gamblet calls reject a bad q, patch radius or NULL pointer
    before any device work."""
    _, L = _lib()
    p = ctypes.c_void_p(16)
    assert L.gbl_mass_inverse(1, 3, p, None) == -1
    assert b"q must be" in L.gbl_last_error(None)
    assert L.gbl_mass_inverse(6, 0, p, None) == -1
    assert L.gbl_mass_inverse(6, 5, p, None) == -1
    assert b"rho_q" in L.gbl_last_error(None)
    assert L.gbl_mass_inverse(6, 3, None, None) == -1
    assert L.gbl_level_q_gamblets(6, 3, p, None, None) == -1
    assert L.gbl_level_q_load(6, 3, p, None, p, None) == -1
    assert L.gbl_level_q_load(6, 3, p, p, p, None) == -1
    assert b"overlap" in L.gbl_last_error(None)
    assert L.gbl_level_q_operator(13, 3, p, p, p, None) == -1
    assert L.gbl_level_q_operator(6, 3, None, p, p, None) == -1
    assert L.gbl_level_q_to_nodal(6, 3, p, p, p, None) == -1


def test_level_q_mass_option_validated():
    P, L = _lib()
    o = P.make_opts(level_q_mass=5)
    assert L.gbl_workspace_bytes(6, ctypes.byref(o), ctypes.byref(ctypes.c_size_t())) == -1
    assert b"level_q_mass" in L.gbl_last_error(None)
    o = P.make_opts(level_q_mass=2, inner="cg")
    assert L.gbl_workspace_bytes(6, ctypes.byref(o), ctypes.byref(ctypes.c_size_t())) == -1
    o = P.make_opts(level_q_mass=3)
    assert L.gbl_workspace_bytes(2, ctypes.byref(o), ctypes.byref(ctypes.c_size_t())) == -1   # 2^2 - 1 < 7
    assert P.workspace_bytes(6, P.make_opts(level_q_mass=3)) > P.workspace_bytes(6, P.make_opts())


def test_rho_coarse_option_validated():
    P, L = _lib()
    o = P.make_opts(rho_coarse=5)
    assert L.gbl_workspace_bytes(6, ctypes.byref(o), ctypes.byref(ctypes.c_size_t())) == -1
    assert b"rho_coarse" in L.gbl_last_error(None)
    o = P.make_opts(rho_coarse=-1)
    assert L.gbl_workspace_bytes(6, ctypes.byref(o), ctypes.byref(ctypes.c_size_t())) == -1
    # a smaller radius below the finest level needs less workspace
    assert P.workspace_bytes(8, P.make_opts(rho=3, rho_coarse=1)) < P.workspace_bytes(8, P.make_opts(rho=3))


def test_noalloc_compression_rejects_bad_sizes():
    """gbl_compress_noalloc validates on the host before touching the device."""
    _, L = _lib()
    thr = ctypes.c_double(0.0)
    dummy = ctypes.c_void_p(4096)   # never dereferenced: every call below fails validation first
    assert L.gbl_compress_noalloc(None, 10, 1, ctypes.byref(thr), None) == -1
    assert L.gbl_compress_noalloc(dummy, 0, 1, ctypes.byref(thr), None) == -1
    assert L.gbl_compress_noalloc(dummy, 1 << 32, 1, ctypes.byref(thr), None) == -1
    assert b"count" in L.gbl_last_error(None)


def test_exact_options_validated():
    """The exact hierarchy needs FP64 and 2 <= q <= 7; the Example 5.1 mesh and
    nodal sources exist only with it."""
    P, L = _lib()
    sz = ctypes.c_size_t()
    bad = [P.make_opts(precision="mixed", exact=True), P.make_opts(precision="fp64", geometry=1),
           P.make_opts(precision="fp64", source="nodal")]
    for o in bad:
        assert L.gbl_workspace_bytes(6, ctypes.byref(o), ctypes.byref(sz)) == -1
    o = P.make_opts(precision="fp64", exact=True)
    assert L.gbl_workspace_bytes(8, ctypes.byref(o), ctypes.byref(sz)) == -1
    assert b"q <= 7" in L.gbl_last_error(None)
    assert L.gbl_workspace_bytes(6, ctypes.byref(P.make_opts(precision="fp64", w_kind=1)), ctypes.byref(sz)) == -1
    assert b"Construction 4.11" in L.gbl_last_error(None)
    assert P.workspace_bytes(6, P.make_opts(precision="fp64", exact=True, w_kind=1)) > 0
    for field, value in (("exact", 2), ("geometry", 2), ("source", 2), ("w_kind", 2)):
        o = P.make_opts(precision="fp64", exact=True)
        setattr(o, field, value)
        assert L.gbl_workspace_bytes(6, ctypes.byref(o), ctypes.byref(sz)) == -1
    g0 = P.workspace_bytes(6, P.make_opts(precision="fp64", exact=True))
    g1 = P.workspace_bytes(6, P.make_opts(precision="fp64", exact=True, geometry=1))
    # the dense level-6 stiffness matrix alone: 3969^2 (geometry 0) and 4096^2 (geometry 1) doubles
    assert g0 > 3969 ** 2 * 8 and g1 > 4096 ** 2 * 8 and g1 > g0


def test_three_dimensional_options_validated():
    """dim 3 exists for the exact hierarchy only, up to q = 4 (16^3 cells)."""
    P, L = _lib()
    sz = ctypes.c_size_t()
    assert L.gbl_workspace_bytes(3, ctypes.byref(P.make_opts(precision="fp64", dim=3)), ctypes.byref(sz)) == -1
    assert L.gbl_workspace_bytes(3, ctypes.byref(P.make_opts(precision="fp64", exact=True, dim=4)),
                                 ctypes.byref(sz)) == -1
    assert L.gbl_workspace_bytes(5, ctypes.byref(P.make_opts(precision="fp64", exact=True, dim=3)),
                                 ctypes.byref(sz)) == -1
    assert b"q <= 4" in L.gbl_last_error(None)
    # q = 4: the dense level-4 stiffness alone is 3375^2 doubles
    assert P.workspace_bytes(4, P.make_opts(precision="fp64", exact=True, dim=3)) > 3375 ** 2 * 8


def test_tensor_option_validated():
    P, L = _lib()
    sz = ctypes.c_size_t()
    assert L.gbl_workspace_bytes(5, ctypes.byref(P.make_opts(precision="fp64", tensor=True)), ctypes.byref(sz)) == -1
    assert L.gbl_workspace_bytes(3, ctypes.byref(P.make_opts(precision="fp64", exact=True, tensor=True, dim=3)),
                                 ctypes.byref(sz)) == -1
    o = P.make_opts(precision="fp64", exact=True, tensor=True)
    assert P.workspace_bytes(5, o) > P.workspace_bytes(5, P.make_opts(precision="fp64", exact=True))
