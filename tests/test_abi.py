"""Host-side checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects invalid problems before any device work."""

import ctypes as C
import re

import numpy as np
import pytest

import synth
import paper_2504_05604_amd as pkg
from paper_2504_05604_amd import _lib


def declared_functions():
    text = open("include/topo.h").read()
    return sorted(set(re.findall(r"\b(topo_[a-z_A-Z]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTED)


def test_default_opts():
    o = pkg.default_opts()
    assert o.precision == pkg.PREC_FP64 and o.precond == pkg.PRECOND_MG
    assert o.rtol == 1e-8 and o.oc_tol == 1e-12 and o.warm_start == 3
    assert o.cheb_degree == 1 and o.cheb_degree_coarse == 4
    assert o.ku_kernel == pkg.KU_AUTO and o.ku_shape == -1 and o.coarse_tail_nodes == 0
    assert o.mg_max_coarse_dof == 1500 and o.coarse_refresh == 1
    assert o.group_launch == 1 and list(o.cheb_degree_level) == [0] * 8 and o.cheb_upper == 1.0


def setup_status(p, vol_mode=0, **opt):
    lib = pkg.load()
    mask = None if p.mask is None else np.ascontiguousarray(p.mask, np.int8)
    fixed = np.ascontiguousarray(p.fixed_dofs, np.int64)
    f = np.ascontiguousarray(p.f, np.float64)
    pc = _lib.Problem_C(p.nelx, p.nely, p.nelz, p.E0, p.Emin, p.nu, p.penal, p.rmin, p.volfrac,
                        p.move, p.eta, 0, vol_mode,
                        None if mask is None else mask.ctypes.data_as(C.POINTER(C.c_int8)),
                        fixed.ctypes.data_as(C.POINTER(C.c_int64)), fixed.size,
                        f.ctypes.data_as(C.POINTER(C.c_double)))
    o = pkg.default_opts(**opt)
    h = C.c_void_p()
    st = lib.topo_setup(C.byref(pc), C.byref(o), None, C.byref(h))
    return st, lib.topo_last_error().decode(), h


@pytest.mark.parametrize("field,value,msg", [
    ("nelx", 0, "grid sizes"), ("rmin", -1.0, "rmin"), ("volfrac", 1.5, "volfrac"),
    ("Emin", 0.0, "Emin"), ("nu", 0.5, "nu"), ("move", 0.0, "move"), ("penal", 0.5, "penal"),
])
def test_setup_rejects_invalid_scalars(field, value, msg):
    p = synth.config_small()
    setattr(p, field, value)
    if field == "nelx":
        p.f = np.zeros(3 * (1) * (p.nely + 1) * (p.nelz + 1))
    st, err, h = setup_status(p)
    assert st == _lib.TOPO_EINVAL and msg in err
    assert not h.value


def test_setup_rejects_bad_mask_and_fixed_dofs():
    p = synth.config_small()
    p.mask = np.zeros(p.nel, np.int8)
    p.mask[3] = 5
    st, err, _ = setup_status(p)
    assert st == _lib.TOPO_EINVAL and "mask value" in err
    p = synth.config_small()
    p.fixed_dofs = np.array([0, 1, 2, p.ndof], np.int64)
    st, err, _ = setup_status(p)
    assert st == _lib.TOPO_EINVAL
    p = synth.config_small()
    p.fixed_dofs = p.fixed_dofs[:3]
    st, err, _ = setup_status(p)
    assert st == _lib.TOPO_EINVAL and "rigid-body" in err
    p = synth.config_small()
    p.mask = np.ones(p.nel, np.int8)
    st, err, _ = setup_status(p)
    assert st == _lib.TOPO_EINVAL and "no design element" in err


def test_setup_rejects_bad_volume_modes():
    p = synth.config_small()
    st, err, _ = setup_status(p, vol_mode=2)
    assert st == _lib.TOPO_EINVAL and "vol_mode" in err
    # fixed solids alone above volfrac * nel leave the design elements no volume
    p.mask = np.zeros(p.nel, np.int8)
    p.mask[: int(0.5 * p.nel)] = 2
    p.volfrac = 0.4
    st, err, _ = setup_status(p, vol_mode=1)
    assert st == _lib.TOPO_EINVAL and "fixed-solid" in err


def test_setup_rejects_bad_options():
    p = synth.config_small()
    for kw, msg in [({"cheb_degree": 0}, "cheb_degree"), ({"rtol": 0.0}, "rtol"),
                    ({"precond": 9}, "preconditioner"), ({"precision": 7}, "precision"),
                    ({"ku_kernel": 3}, "ku_kernel"), ({"ku_shape": 4}, "ku_shape"),
                    ({"ku_shape": 5}, "ku_shape"), ({"ku_shape": 15}, "ku_shape"),
                    ({"ku_shape": -2}, "ku_shape"), ({"coarse_refresh": 0}, "coarse_refresh"),
                    ({"cheb_degree_coarse": -1}, "cheb_degree_coarse"), ({"cheb_degree_coarse": 17}, "cheb_degree_coarse"),
                    ({"group_launch": 2}, "group_launch"), ({"group_launch": -1}, "group_launch"),
                    ({"autotune": 3}, "autotune"), ({"autotune": -1}, "autotune"),
                    ({"cheb_upper": 0.0}, "cheb_upper"), ({"cheb_upper": 1.5}, "cheb_upper")]:
        st, err, _ = setup_status(p, **kw)
        assert st == _lib.TOPO_EINVAL and msg in err, (kw, err)


def test_batch_and_network_entry_points_reject_invalid_arguments():
    lib = pkg.load()
    h = C.c_void_p()
    o = pkg.default_opts()
    st = lib.topo_setup_batch(None, 3, C.byref(o), 0, C.byref(h))
    assert st == _lib.TOPO_EINVAL and "at least one problem" in lib.topo_last_error().decode()
    p = synth.config_small()
    pc, keep = _lib._problem_c(p)
    arr = (_lib.Problem_C * 1)(pc)
    st = lib.topo_setup_batch(arr, 1, C.byref(o), 100, C.byref(h))
    assert st == _lib.TOPO_EINVAL and "n_threads" in lib.topo_last_error().decode()
    st = lib.topo_iterate_batch(None, None, 1, None)
    assert st == _lib.TOPO_EINVAL
    bad = (C.c_int32 * 3)(16, 0, 64)
    st = lib.topo_nn_create(bad, None, C.byref(h))
    assert st == _lib.TOPO_EINVAL and "channel" in lib.topo_last_error().decode()
    assert lib.topo_set_nn(None, None) == _lib.TOPO_EINVAL


def test_default_train_opts():
    t = pkg.default_train_opts()
    assert (t.epochs, t.batch, t.lr, t.beta1, t.beta2, t.eps, t.loss) == (10, 4, 1e-3, 0.9, 0.999, 1e-8, pkg.LOSS_REL)
    o = pkg.default_opts()
    assert o.nn_max_iters == 200 and o.autotune == 0


def test_noalloc_oc_update_validates_before_device_work():
    lib = pkg.load()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    args = [fake, fake, fake, fake, 0.2, 0.5, 10.0, 1e-12, None, C.c_void_p(0x2000), None]
    assert lib.topo_oc_update_noalloc(0, *args) == _lib.TOPO_EINVAL
    assert "nel" in lib.topo_last_error().decode()
    bad = list(args)
    bad[4] = 0.0
    assert lib.topo_oc_update_noalloc(10, *bad) == _lib.TOPO_EINVAL
    bad = list(args)
    bad[6] = -1.0
    assert lib.topo_oc_update_noalloc(10, *bad) == _lib.TOPO_EINVAL
    assert "target" in lib.topo_last_error().decode()
    bad = list(args)
    bad[9] = fake  # d_xnew aliasing d_x
    assert lib.topo_oc_update_noalloc(10, *bad) == _lib.TOPO_EINVAL
    assert lib.topo_oc_update_noalloc(10, None, *args[1:]) == _lib.TOPO_EINVAL
