"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and
rejects invalid arguments before touching a device (so these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2509_21039_amd as hfk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "hfk.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hfk_status|const char \*)\s*(hfk_\w+)\s*\(", src, re.M)))


def test_header_declares_entry_points():
    names = _declared_symbols()
    for must in ("hfk_fock", "hfk_fock_grad", "hfk_fock_batched", "hfk_workspace_bytes",
                 "hfk_batched_workspace_bytes", "hfk_read_stats", "hfk_tune", "hfk_last_error",
                 "hfk_fock_atoms", "hfk_workspace_bytes_atoms", "hfk_fock_grad_atoms",
                 "hfk_fock_batched_atoms", "hfk_batched_workspace_bytes_atoms", "hfk_scf",
                 "hfk_scf_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = hfk.lib()
    for name in _declared_symbols():
        assert hasattr(L, name), name
    assert hfk.version().startswith("hfk")


def _fock_raw(n=4, ngauss=3, exps=(6.36242139, 1.158923, 0.31364979), coefs=(0.15432897, 0.53532814, 0.44463454),
              xyz=1, dens=1, tau=1e-10, prec=0, strat=0, fock=1, e2=1, ws=256, wsb=1 << 40):
    e = np.ascontiguousarray(exps, dtype=np.float64)
    c = np.ascontiguousarray(coefs, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    return hfk.lib().hfk_fock(n, xyz, ngauss, e.ctypes.data_as(dp), c.ctypes.data_as(dp), dens, tau, prec, strat,
                              fock, e2, ws, wsb, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0), "natoms"),
    (dict(n=-5), "natoms"),
    (dict(ngauss=0, exps=(1.0,), coefs=(1.0,)), "ngauss"),
    (dict(ngauss=9, exps=(1.0,) * 9, coefs=(1.0,) * 9), "ngauss"),
    (dict(xyz=None), "xyz"),
    (dict(dens=None), "dens"),
    (dict(exps=(1.0, -2.0, 3.0)), "exps"),
    (dict(exps=(1.0, float("nan"), 3.0)), "exps"),
    (dict(coefs=(1.0, float("inf"), 3.0)), "coefs"),
    (dict(tau=-1.0), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(prec=7), "precision"),
    (dict(strat=9), "strategy"),
    (dict(fock=None), "fock"),
    (dict(e2=None), "e2"),
    (dict(ws=None), "workspace"),
    (dict(ws=257), "aligned"),
])
def test_fock_rejects_invalid_arguments(kw, msg):
    st = _fock_raw(**kw)
    assert st == hfk.HFK_EINVAL
    assert msg in hfk.lib().hfk_last_error().decode()


def _grad_raw(n=4, xyz=1, dens=1, g_e2=1, g_fock=None, fock_in=None, d_xyz=1, d_dens=None, ws=256):
    e = np.ascontiguousarray((6.36242139, 1.158923, 0.31364979), dtype=np.float64)
    c = np.ascontiguousarray((0.15432897, 0.53532814, 0.44463454), dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    return hfk.lib().hfk_fock_grad(n, xyz, 3, e.ctypes.data_as(dp), c.ctypes.data_as(dp), dens, 1e-10, 0, g_e2,
                                   g_fock, fock_in, d_xyz, d_dens, None, ws, 1 << 40, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0), "natoms"),
    (dict(g_e2=None), "g_e2"),
    (dict(d_xyz=None), "d_xyz"),
    (dict(d_dens=1), "fock_in"),
    (dict(d_dens=1, g_fock=1), "fock_in"),
    (dict(ws=None), "workspace"),
])
def test_fock_grad_rejects_invalid_arguments(kw, msg):
    st = _grad_raw(**kw)
    assert st == hfk.HFK_EINVAL
    assert msg in hfk.lib().hfk_last_error().decode()


def test_workspace_bytes_validation():
    out = ctypes.c_size_t(0)
    L = hfk.lib()
    assert L.hfk_workspace_bytes(0, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes(10, 9, 0, 0, ctypes.byref(out)) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes(10, 3, 5, 0, ctypes.byref(out)) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes(10, 3, 0, 0, None) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes(10, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_OK
    small = out.value
    assert L.hfk_workspace_bytes(100, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_OK
    assert out.value > small
    assert L.hfk_workspace_bytes(100000, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_EUNSUPPORTED


def test_python_layer_raises_hfkerror():
    with pytest.raises(hfk.HfkError) as ei:
        hfk.workspace_bytes(0)
    assert ei.value.status == hfk.HFK_EINVAL


def test_read_stats_null_arguments():
    assert hfk.lib().hfk_read_stats(None, None, None) == hfk.HFK_EINVAL


def test_load_tuning_rejects_missing_and_foreign_files(tmp_path):
    with pytest.raises(hfk.HfkError):
        hfk.load_tuning(str(tmp_path / "missing.json"))
    bad = tmp_path / "bad.json"
    bad.write_text('{"something": 1}')
    with pytest.raises(hfk.HfkError):
        hfk.load_tuning(str(bad))
    # the previous format, keyed by a size class, is not read
    old = tmp_path / "old.json"
    old.write_text('{"format": "hfk-tuning-1", "entries": [{"precision": 0, "size_class": 1, "strategy": 1, '
                   '"variant": 1, "gpc": 4}]}')
    with pytest.raises(hfk.HfkError):
        hfk.load_tuning(str(old))
    entry = ('{"arch": "gfx950", "precision": 0, "size_bucket": 9, "strategy": %d, "variant": 1, "gpc": 4, '
             '"tile_items": %d, "group_bras": %d, "ket_copies": 0}')
    for strat, tile, gb in ((7, 4, 1024), (3, 4, 1024), (2, 0, 1024), (2, 17, 1024), (2, 4, 1000), (2, 4, 8192)):
        worse = tmp_path / "worse.json"
        worse.write_text('{"format": "hfk-tuning-2", "entries": [%s], "batched": []}' % (entry % (strat, tile, gb)))
        with pytest.raises(hfk.HfkError):
            hfk.load_tuning(str(worse))
    for gpc, items, owned, w in ((0, 0, -1, 8), (5, 0, -1, 8), (2, 2000, -1, 8), (2, 0, 0, 8), (2, 0, -5, 8),
                                 (2, 0, -1, 6)):
        worse = tmp_path / "worse_b.json"
        worse.write_text('{"format": "hfk-tuning-2", "entries": [], "batched": [{"arch": "gfx950", "precision": 1, '
                         '"gpc": %d, "block_items": %d, "owned_bound": %d, "waves": %d}]}' % (gpc, items, owned, w))
        with pytest.raises(hfk.HfkError):
            hfk.load_tuning(str(worse))


def test_load_tuning_accepts_its_format(tmp_path):
    good = tmp_path / "good.json"
    good.write_text('{\n  "format": "hfk-tuning-2",\n  "entries": [\n'
                    '    {"arch": "gfx950", "precision": 0, "size_bucket": 9, "strategy": 2, "variant": 1, "gpc": 4, '
                    '"tile_items": 8, "group_bras": 2048, "ket_copies": 8},\n'
                    '    {"arch": "gfx942", "precision": 1, "size_bucket": 10, "strategy": 1, "variant": 0, "gpc": 6, '
                    '"tile_items": 4, "group_bras": 256, "ket_copies": 0}\n  ],\n'
                    '  "batched": [\n    {"arch": "gfx950", "precision": 1, "gpc": 3, "block_items": 32, '
                    '"owned_bound": 65536, "waves": 4}\n  ]\n}\n')
    hfk.load_tuning(str(good))
    hfk.clear_tuning()


def test_set_config_validation():
    L = hfk.lib()
    assert L.hfk_set_config(2, 0) == hfk.HFK_EINVAL
    assert L.hfk_set_config(-1, 9) == hfk.HFK_EINVAL
    assert L.hfk_set_config(-1, 0) == hfk.HFK_OK


def test_set_shape_validation():
    L = hfk.lib()
    for tile, gb, kc in ((17, 0, -1), (-1, 0, -1), (4, 1000, -1), (4, 128, -1), (4, 8192, -1), (4, 1024, -2),
                         (4, 1024, 1025)):
        assert L.hfk_set_shape(tile, gb, kc) == hfk.HFK_EINVAL, (tile, gb, kc)
    for tile, gb, kc in ((1, 256, 0), (16, 4096, 1024), (8, 512, 8)):
        assert L.hfk_set_shape(tile, gb, kc) == hfk.HFK_OK
    assert L.hfk_set_shape(0, 0, -1) == hfk.HFK_OK


def test_set_batched_config_validation():
    L = hfk.lib()
    for gpc, items, owned, w in ((5, 0, 0, 0), (-1, 0, 0, 0), (2, 1025, 0, 0), (2, -1, 0, 0), (2, 0, -2, 0),
                                 (2, 0, 0, 2), (2, 0, 0, 16)):
        assert L.hfk_set_batched_config(gpc, items, owned, w) == hfk.HFK_EINVAL, (gpc, items, owned, w)
    for gpc, items, owned, w in ((4, 1024, 1 << 18, 8), (1, 8, -1, 4)):
        assert L.hfk_set_batched_config(gpc, items, owned, w) == hfk.HFK_OK
    assert L.hfk_set_batched_config(0, 0, 0, 0) == hfk.HFK_OK


def test_set_debug_validation():
    L = hfk.lib()
    for tol in (-1e-12, float("nan"), float("inf")):
        assert L.hfk_set_debug(1, tol) == hfk.HFK_EINVAL, tol
    assert L.hfk_set_debug(1, 0.0) == hfk.HFK_OK
    assert L.hfk_set_debug(0, 1e-12) == hfk.HFK_OK


def test_last_stats_needs_a_build_on_this_thread():
    """No build call has run on a fresh thread: hfk_last_stats refuses (host check, no HIP call)."""
    import threading
    out = {}

    def probe():
        st = hfk.HfkStats()
        out["status"] = hfk.lib().hfk_last_stats(ctypes.byref(st))
        out["null"] = hfk.lib().hfk_last_stats(None)

    t = threading.Thread(target=probe)
    t.start()
    t.join()
    assert out["status"] == hfk.HFK_EINVAL and out["null"] == hfk.HFK_EINVAL


def test_batched_pair_limit():
    """A batch above the pair limit of one call (its ket-table buffer offsets stay below
    2^31) is refused on the host: 2501 molecules of 128 atoms hold 20.6M pairs, 5000 hold
    41.3M."""
    import numpy as np
    L = hfk.lib()
    out = ctypes.c_size_t(0)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ok = np.arange(0, 128 * 2502, 128, dtype=np.int64)
    assert L.hfk_batched_workspace_bytes(len(ok) - 1, ok.ctypes.data_as(i64p), 6, 0, 1, ctypes.byref(out)) == hfk.HFK_OK
    big = np.arange(0, 128 * 5001, 128, dtype=np.int64)
    assert (L.hfk_batched_workspace_bytes(len(big) - 1, big.ctypes.data_as(i64p), 6, 0, 1, ctypes.byref(out))
            == hfk.HFK_EUNSUPPORTED)
    assert "pairs" in hfk.lib().hfk_last_error().decode()


def test_batched_validation():
    import numpy as np
    L = hfk.lib()
    out = ctypes.c_size_t(0)
    i64p = ctypes.POINTER(ctypes.c_int64)
    off = np.array([0, 3, 3], dtype=np.int64)            # empty molecule
    assert L.hfk_batched_workspace_bytes(2, off.ctypes.data_as(i64p), 3, 1, 1, ctypes.byref(out)) == hfk.HFK_EINVAL
    off = np.array([1, 3], dtype=np.int64)               # must start at 0
    assert L.hfk_batched_workspace_bytes(1, off.ctypes.data_as(i64p), 3, 1, 1, ctypes.byref(out)) == hfk.HFK_EINVAL
    off = np.array([0, 200], dtype=np.int64)             # above the LDS limit
    assert L.hfk_batched_workspace_bytes(1, off.ctypes.data_as(i64p), 3, 1, 1, ctypes.byref(out)) == hfk.HFK_EUNSUPPORTED
    off = np.array([0, 4, 9], dtype=np.int64)
    assert L.hfk_batched_workspace_bytes(2, off.ctypes.data_as(i64p), 3, 1, 1, ctypes.byref(out)) == hfk.HFK_OK
    assert out.value > 0


def _atoms_raw(n=4, g=3, exps=None, coefs=None, xyz=1, dens=1, tau=1e-10, prec=0, strat=0, fock=1, e2=1, ws=256):
    e = np.ascontiguousarray(np.tile([6.36242139, 1.158923, 0.31364979], (n, 1)) if exps is None else exps,
                             dtype=np.float64)
    c = np.ascontiguousarray(np.tile([0.15432897, 0.53532814, 0.44463454], (n, 1)) if coefs is None else coefs,
                             dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    return hfk.lib().hfk_fock_atoms(n, xyz, g, e.ctypes.data_as(dp), c.ctypes.data_as(dp), dens, tau, prec,
                                    strat, fock, e2, ws, 1 << 40, None)


def _bad_row(col, value, atom=2, which="exps"):
    a = np.tile([6.36242139, 1.158923, 0.31364979] if which == "exps" else [0.15432897, 0.53532814, 0.44463454],
                (4, 1))
    a[atom, col] = value
    return {which: a}


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0), "natoms"),
    (_bad_row(1, -1.0), "atom 2"),
    (_bad_row(0, 0.0, atom=3), "atom 3"),
    (_bad_row(2, float("nan"), atom=1), "atom 1"),
    (_bad_row(1, float("inf"), which="coefs"), "atom 2"),
    (dict(tau=-1.0), "tau"),
    (dict(prec=3), "precision"),
    (dict(strat=9), "strategy"),
    (dict(fock=None), "fock"),
    (dict(ws=None), "workspace"),
    (dict(ws=300), "aligned"),
])
def test_fock_atoms_rejects_invalid_arguments(kw, msg):
    """Every atom's row is validated on the host; the message names the atom."""
    assert _atoms_raw(**kw) == hfk.HFK_EINVAL
    assert msg in hfk.lib().hfk_last_error().decode()


def test_workspace_bytes_atoms_validation():
    out = ctypes.c_size_t(0)
    L = hfk.lib()
    assert L.hfk_workspace_bytes_atoms(0, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes_atoms(10, 9, 0, 0, ctypes.byref(out)) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes_atoms(10, 3, 4, 0, ctypes.byref(out)) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes_atoms(10, 3, 0, 0, None) == hfk.HFK_EINVAL
    assert L.hfk_workspace_bytes_atoms(100000, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_EUNSUPPORTED
    assert L.hfk_workspace_bytes_atoms(5000, 3, 0, 1, ctypes.byref(out)) == hfk.HFK_EUNSUPPORTED
    assert L.hfk_workspace_bytes_atoms(300, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_OK
    atoms = out.value
    assert L.hfk_workspace_bytes(300, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_OK
    assert atoms > out.value   # the per-atom tables come on top of the one-basis layout
    assert L.hfk_workspace_bytes_atoms(300, 3, 0, 1, ctypes.byref(out)) == hfk.HFK_OK
    assert out.value > atoms   # and the gradient's tables on top of those


def test_fock_grad_atoms_rejects_bad_rows():
    e = np.tile([6.36242139, 1.158923, 0.31364979], (4, 1))
    c = np.tile([0.15432897, 0.53532814, 0.44463454], (4, 1))
    e[3, 2] = -0.5
    dp = ctypes.POINTER(ctypes.c_double)
    st = hfk.lib().hfk_fock_grad_atoms(4, 1, 3, e.ctypes.data_as(dp), c.ctypes.data_as(dp), 1, 1e-10, 0, 1, None,
                                       None, 1, None, None, 256, 1 << 40, None)
    assert st == hfk.HFK_EINVAL
    assert "atom 3" in hfk.lib().hfk_last_error().decode()


def test_fock_batched_atoms_rejects_bad_rows():
    off = np.array([0, 2, 5], dtype=np.int64)
    e = np.tile([6.36242139, 1.158923, 0.31364979], (5, 1))
    c = np.tile([0.15432897, 0.53532814, 0.44463454], (5, 1))
    c[4, 0] = float("nan")
    dp = ctypes.POINTER(ctypes.c_double)
    st = hfk.lib().hfk_fock_batched_atoms(2, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, 3,
                                          e.ctypes.data_as(dp), c.ctypes.data_as(dp), 1, 1e-10, 0, 1, 1, None,
                                          256, 1 << 40, None)
    assert st == hfk.HFK_EINVAL
    assert "atom 4" in hfk.lib().hfk_last_error().decode()
    out = ctypes.c_size_t(0)
    L = hfk.lib()
    p64 = ctypes.POINTER(ctypes.c_int64)
    assert L.hfk_batched_workspace_bytes(2, off.ctypes.data_as(p64), 3, 1, 1, ctypes.byref(out)) == hfk.HFK_OK
    one = out.value
    assert L.hfk_batched_workspace_bytes_atoms(2, off.ctypes.data_as(p64), 3, 1, 1, ctypes.byref(out)) == hfk.HFK_OK
    assert out.value > one


def test_deterministic_strategy_size_limit():
    """The deterministic strategy is refused above 1024 atoms before any device work; strategy
    values past it are invalid."""
    assert _fock_raw(n=1025, strat=3) == hfk.HFK_EUNSUPPORTED
    assert "deterministic" in hfk.lib().hfk_last_error().decode()
    assert _fock_raw(strat=4) == hfk.HFK_EINVAL
    assert _atoms_raw(n=1100, strat=3) == hfk.HFK_EUNSUPPORTED


def _scf_raw(n=4, charges=None, nocc=2, max_iter=50, e_tol=1e-10, d_tol=1e-7, dens=1, strat=0, e=None):
    ee = np.ascontiguousarray(np.tile([6.36242139, 1.158923, 0.31364979], (n, 1)) if e is None else e)
    cc = np.ascontiguousarray(np.tile([0.15432897, 0.53532814, 0.44463454], (n, 1)))
    Z = np.ascontiguousarray(np.full(n, 2.0) if charges is None else charges, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    E = ctypes.c_double(0.0)
    it = ctypes.c_int32(0)
    cv = ctypes.c_int32(0)
    return hfk.lib().hfk_scf(n, 1, Z.ctypes.data_as(dp), 3, ee.ctypes.data_as(dp), cc.ctypes.data_as(dp), nocc,
                             1e-10, 0, strat, max_iter, e_tol, d_tol, dens, 0, None, ctypes.byref(E),
                             ctypes.byref(it), ctypes.byref(cv), 256, 1 << 40, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(charges=[2.0, -1.0, 2.0, 2.0]), "charges"),
    (dict(charges=[2.0, float("nan"), 2.0, 2.0]), "charges"),
    (dict(nocc=5), "nocc"),
    (dict(nocc=-1), "nocc"),
    (dict(max_iter=0), "max_iter"),
    (dict(e_tol=0.0), "e_tol"),
    (dict(d_tol=float("inf")), "d_tol"),
    (dict(dens=None), "dens"),
    (dict(strat=7), "strategy"),
])
def test_scf_rejects_invalid_arguments(kw, msg):
    assert _scf_raw(**kw) == hfk.HFK_EINVAL
    assert msg in hfk.lib().hfk_last_error().decode()


def test_scf_workspace_bytes():
    out = ctypes.c_size_t(0)
    L = hfk.lib()
    assert L.hfk_scf_workspace_bytes(0, 3, 0, ctypes.byref(out)) == hfk.HFK_EINVAL
    assert L.hfk_scf_workspace_bytes(100, 3, 0, ctypes.byref(out)) == hfk.HFK_OK
    small = out.value
    assert L.hfk_workspace_bytes_atoms(100, 3, 0, 0, ctypes.byref(out)) == hfk.HFK_OK
    assert small > out.value + 10 * 100 * 100 * 8   # the SCF matrices come on top of the Fock layout
