"""Host-side checks of the C ABI (no GPU compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mehdg.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mehdg_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mehdg_create", "mehdg_destroy", "mehdg_assemble", "mehdg_condense",
                     "mehdg_recover", "mehdg_status"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2507_22195_amd import mehdg
    if not os.path.exists(mehdg.LIB_PATH):
        pytest.skip("libmehdg.so not built")
    lib = ctypes.CDLL(mehdg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_are_synchronous():
    """Calls with bad arguments return EINVAL without touching a device."""
    from paper_2507_22195_amd import mehdg
    if not os.path.exists(mehdg.LIB_PATH):
        pytest.skip("libmehdg.so not built")
    lib = mehdg.load()
    out = (ctypes.c_int64 * 5)()
    assert lib.mehdg_sizes(0, out) == 1 and lib.mehdg_sizes(5, out) == 1
    assert lib.mehdg_sizes(2, out) == 0 and list(out) == [125, 25, 625, 1875, 750]
    assert lib.mehdg_sizes(4, out) == 0 and list(out) == [729, 81, 3645, 10935, 2430]
    assert lib.mehdg_create(None, None, None) == 1
    h = (ctypes.c_double * 3)(0.1, 0.1, -0.1)     # negative size
    mesh = mehdg.Mesh(1, 2, 0, ctypes.cast(h, ctypes.POINTER(ctypes.c_double)))
    prm = mehdg.make_params(dict(gamma=1.4, mu=0, kappa=0, lam=0, sigma_vis=[0] * 5, alpha_t=0,
                                 alpha_ps=0, logmean_eps=1e-4, flux=0, viscous=0))
    handle = ctypes.c_void_p()
    assert lib.mehdg_create(ctypes.byref(mesh), ctypes.byref(prm), ctypes.byref(handle)) == 1
    assert handle.value is None
    mesh = mehdg.Mesh(1, 7, 0, ctypes.cast(h, ctypes.POINTER(ctypes.c_double)))   # bad degree
    assert lib.mehdg_create(ctypes.byref(mesh), ctypes.byref(prm), ctypes.byref(handle)) == 1
    assert lib.mehdg_assemble(None, *([None] * 8), 0, None) == 1
    assert lib.mehdg_condense(None, 0, None, None, None) == 1
    assert lib.mehdg_condense(None, 3, None, None, None) == 1
    assert lib.mehdg_recover(None, None, None, None, None, None) == 1
    assert lib.mehdg_status(None, None, None) == 1
    assert lib.mehdg_jvp(None, *([None] * 6), None) == 1
    assert lib.mehdg_vjp(None, *([None] * 6), None) == 1
    assert lib.mehdg_condense_rhs(None, None, None, None, None) == 1
    # batches: bad degree or empty mesh before any device work, NULL handles
    handle = ctypes.c_void_p()
    deg = (ctypes.c_int32 * 2)(2, 5)
    hh = (ctypes.c_double * 6)(0.1, 0.1, 0.1, 0.1, 0.1, 0.1)
    bm = mehdg.BatchMesh(2, deg, ctypes.cast(hh, ctypes.POINTER(ctypes.c_double)), None, 0, 0, 0)
    assert lib.mehdg_batch_create(ctypes.byref(bm), ctypes.byref(prm), ctypes.byref(handle)) == 1
    assert handle.value is None
    bm = mehdg.BatchMesh(0, deg, ctypes.cast(hh, ctypes.POINTER(ctypes.c_double)), None, 0, 0, 0)
    assert lib.mehdg_batch_create(ctypes.byref(bm), ctypes.byref(prm), ctypes.byref(handle)) == 1
    assert lib.mehdg_batch_create(None, None, None) == 1
    assert lib.mehdg_batch_destroy(None) == 1
    assert lib.mehdg_batch_layout(None, 0, None, None) == 1
    assert lib.mehdg_batch_groups(None, None, None, None, None, None) == 1
    assert lib.mehdg_batch_assemble_condense(None, 0, *([None] * 9), None) == 1
    assert lib.mehdg_batch_recover(None, *([None] * 7), None) == 1
    assert lib.mehdg_batch_status(None, None, None) == 1
    # tile variants: a list of shapes; NULL contexts and bad sites are EINVAL
    n = ctypes.c_int32()
    assert lib.mehdg_tile_variants(ctypes.byref(n), None) == 0 and n.value >= 1
    shapes = (ctypes.c_int32 * (6 * n.value))()
    assert lib.mehdg_tile_variants(ctypes.byref(n), shapes) == 0
    assert list(shapes[:6]) == [4, 2, 2, 2, 16, 4]          # variant 0: 128 x 64 tiles of 512 threads
    assert lib.mehdg_tile_variants(None, None) == 1
    assert lib.mehdg_set_tile(None, 0, 0) == 1
    assert lib.mehdg_trace_set_inner_precision(None, 0) == 1
    assert lib.mehdg_get_tile(None, 0, ctypes.byref(n)) == 1
    assert lib.mehdg_set_lu_depth(None, 1) == 1
    assert lib.mehdg_get_lu_depth(None, ctypes.byref(n)) == 1


def test_wall_flags_are_checked_before_any_device_work():
    """face_bc entries other than 0 / 1, or walls with T_wall <= 0, are EINVAL."""
    from paper_2507_22195_amd import mehdg
    if not os.path.exists(mehdg.LIB_PATH):
        pytest.skip("libmehdg.so not built")
    lib = mehdg.load()
    h = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    base = dict(gamma=1.4, mu=0, kappa=0, lam=0, sigma_vis=[0] * 5, alpha_t=0, alpha_ps=0, logmean_eps=1e-4,
                flux=0, viscous=0)
    for flags, T_wall in (((0, 0, 0, 0, 2, 0), 1.0), ((0, 0, 0, 0, 1, 0), 0.0), ((0, 0, 0, 0, 1, 0), -1.0)):
        bc = (ctypes.c_uint8 * 6)(*flags)
        mesh = mehdg.Mesh(1, 2, 0, ctypes.cast(h, ctypes.POINTER(ctypes.c_double)),
                          ctypes.cast(bc, ctypes.POINTER(ctypes.c_uint8)))
        prm = mehdg.make_params(dict(base, T_wall=T_wall))
        handle = ctypes.c_void_p()
        assert lib.mehdg_create(ctypes.byref(mesh), ctypes.byref(prm), ctypes.byref(handle)) == 1, (flags, T_wall)
        assert handle.value is None



def test_tet_entry_points_check_arguments_on_the_host():
    """mehdg_tet_*: sizes of the degree-2p lattice; bad degrees, wall flags and
    degenerate macros are EINVAL before any device work."""
    from paper_2507_22195_amd import mehdg
    if not os.path.exists(mehdg.LIB_PATH):
        pytest.skip("libmehdg.so not built")
    lib = mehdg.load()
    out = (ctypes.c_int64 * 5)()
    assert lib.mehdg_tet_sizes(0, out) == 1 and lib.mehdg_tet_sizes(4, out) == 1
    assert lib.mehdg_tet_sizes(3, out) == 0 and list(out) == [84, 28, 420, 1260, 560]
    assert lib.mehdg_tet_sizes(1, out) == 0 and list(out) == [10, 6, 50, 150, 120]
    base = dict(gamma=1.4, mu=0, kappa=0, lam=0, sigma_vis=[0] * 5, alpha_t=0, alpha_ps=0, logmean_eps=1e-4,
                flux=0, viscous=0)
    good = [0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1]
    flat = [0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0]            # fourth vertex in the plane of the others
    cases = [(good, 0, None, 1.0), (good, 4, None, 1.0), (flat, 2, None, 1.0),
             (good, 2, (0, 2, 0, 0), 1.0), (good, 2, (0, 1, 0, 0), 0.0)]
    for X, p, flags, T_wall in cases:
        xs = (ctypes.c_double * 12)(*X)
        bc = None if flags is None else ctypes.cast((ctypes.c_uint8 * 4)(*flags), ctypes.POINTER(ctypes.c_uint8))
        mesh = mehdg.TetMesh(1, p, 0, ctypes.cast(xs, ctypes.POINTER(ctypes.c_double)), bc)
        prm = mehdg.make_params(dict(base, T_wall=T_wall))
        handle = ctypes.c_void_p()
        assert lib.mehdg_tet_create(ctypes.byref(mesh), ctypes.byref(prm), ctypes.byref(handle)) == 1, (p, flags)
        assert handle.value is None
    assert lib.mehdg_tet_create(None, None, None) == 1
    assert lib.mehdg_tet_residual(None, *([None] * 8), None) == 1
    assert lib.mehdg_tet_jvp(None, *([None] * 9), None) == 1
    assert lib.mehdg_tet_assemble(None, *([None] * 7), None) == 1
    assert lib.mehdg_tet_condense(None, None, None, None) == 1
    assert lib.mehdg_tet_recover(None, None, None, None, None, None) == 1
    assert lib.mehdg_tet_vjp(None, None, None, None, None, None) == 1
    assert lib.mehdg_tet_condense_rhs(None, None, None, None, None) == 1
    assert lib.mehdg_tet_status(None, None, None) == 1
    assert lib.mehdg_tet_destroy(None) == 1
