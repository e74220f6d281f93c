"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and
rejects invalid descriptors before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2603_12185_amd import cfsim, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfsim.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cfsim.LIB_PATH):
        from paper_2603_12185_amd import build
        build.build()
    return cfsim.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("cf_model_create", "cf_model_destroy", "cf_model_dims", "cf_step", "cf_rollout",
              "cf_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in cfsim.h but not exported"
    assert set(names) == set(cfsim.SIGNATURES), "binding and header disagree"


def _create(scene):
    d, keep = cfsim.make_desc(scene)
    h = C.c_void_p()
    st = cfsim.load().cf_model_create(C.byref(d), C.byref(h))
    return st, h


@pytest.mark.parametrize("mutate,expect", [
    (lambda s: s.update(condim=2), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(h=0.0), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(h=float("nan")), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(k_user=-0.1), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(solimp=np.array([0.95, 0.9, 0.001, 0.5, 2.0])), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(solimp=np.array([0.9, 0.95, 0.0, 0.5, 2.0])), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(solimp=np.array([0.9, 0.95, 0.001, 1.0, 2.0])), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(solimp=np.array([0.9, 0.95, 0.001, 0.5, 0.5])), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(nworld=0), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(body_mass=np.zeros_like(s["body_mass"])), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(geom_body=np.array([-1, 5], np.int32)), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(geom_type=np.array([0, 7], np.int32)), cfsim.CF_E_INVALID_ARG),
    (lambda s: s.update(body_ipos=np.array([[0.1, 0, 0]])), cfsim.CF_E_INVALID_ARG),
])
def test_invalid_descriptors_rejected(lib, mutate, expect):
    s = scenes.sphere_on_plane()
    s = dict(s)
    mutate(s)
    st, h = _create(s)
    assert st == expect, cfsim.last_error()
    assert not h.value
    assert cfsim.last_error()


def test_unsupported_trees_are_reported(lib):
    """Subtrees must be contiguous in body order and hold at most 32 dofs."""
    b = scenes._Builder(1)
    r0 = b.body(scenes.JNT_HINGE, -1, axis=(0, 1, 0))
    b.body(scenes.JNT_HINGE, -1, axis=(0, 1, 0))
    b.body(scenes.JNT_HINGE, r0, axis=(0, 1, 0))  # child of body 0 after another root
    st, h = _create(b.build())
    assert st == cfsim.CF_E_UNSUPPORTED and not h.value
    assert "contiguous" in cfsim.last_error()
    b = scenes._Builder(1)
    p = -1
    for _ in range(33):
        p = b.body(scenes.JNT_HINGE, p, axis=(0, 1, 0))
    st, h = _create(b.build())
    assert st == cfsim.CF_E_UNSUPPORTED and "32" in cfsim.last_error()


def test_null_arguments(lib):
    assert lib.cf_model_create(None, None) == cfsim.CF_E_INVALID_ARG
    assert lib.cf_step(None, None, None, None, None, None, None, None) == cfsim.CF_E_INVALID_ARG
    assert lib.cf_rollout(None, None, 1, None, None, None, None, None, None, None) == cfsim.CF_E_INVALID_ARG
    assert lib.cf_model_dims(None, None, None, None) == cfsim.CF_E_INVALID_ARG
    lib.cf_model_destroy(None)



def test_impedance_mode_null_model(lib):
    assert lib.cf_model_set_impedance(None, 0) == cfsim.CF_E_INVALID_ARG


def test_actuators_null_model(lib):
    assert lib.cf_model_set_actuators(None, None, None) == cfsim.CF_E_INVALID_ARG
