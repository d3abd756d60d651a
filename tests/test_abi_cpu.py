"""The C-ABI library loads, exports every entry point of include/pic.h, and
rejects bad configurations before touching a GPU.  CPU only."""
import ctypes as C
import os
import re

import pytest

from paper_2104_00642_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"^(?:pic_status|void|const char \*)\s*(pic_\w+)\(", src, re.M)))


def test_exports_every_declared_symbol(piclib):
    names = header_functions()
    assert set(L.EXPORTED) == set(names)
    for n in names:
        assert hasattr(piclib, n), n


def base_cfg(**kw):
    cfg = L.Config(dim=2, n=(64, 64), d=(0.1, 0.1), dt=0.05)
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


@pytest.mark.parametrize("kw,status", [
    (dict(dt=0.1), L.PIC_E_CFL),
    (dict(order=3), L.PIC_E_UNSUPPORTED),
    (dict(dim=1), L.PIC_E_UNSUPPORTED),
    (dict(precision=7), L.PIC_E_UNSUPPORTED),
    (dict(n=(64, 64, 4)), L.PIC_E_ARG),
    (dict(n=(4, 64)), L.PIC_E_ARG),
    (dict(d=(0.0, 0.1)), L.PIC_E_ARG),
    (dict(dt=-1.0), L.PIC_E_ARG),
    (dict(tile=(10, 16)), L.PIC_E_ARG),
    (dict(drift=9), L.PIC_E_ARG),
    (dict(n=(16, 16)), L.PIC_E_UNSUPPORTED),  # grid smaller than the tile window
])
def test_config_validation(piclib, kw, status):
    with pytest.raises(L.PicError) as e:
        L.pic_init(base_cfg(**kw))
    assert e.value.status == status
    assert L.pic_last_error(None)


def test_null_arguments(piclib):
    h = C.c_void_p()
    assert piclib.pic_init(None, C.byref(h)) == L.PIC_E_ARG
    assert piclib.pic_gather_push_deposit(None, None, None, None, None, None) == L.PIC_E_ARG
    assert piclib.pic_yee_step(None, 1, None, None, None) == L.PIC_E_ARG
    assert piclib.pic_sort(None, None, None, None) == L.PIC_E_ARG
    assert piclib.pic_check(None, None, None, None) == L.PIC_E_ARG
    assert piclib.pic_reserve(None, 0) == L.PIC_E_ARG
    assert piclib.pic_deposit_rho(None, None, None, 1, None, None) == L.PIC_E_ARG
    assert piclib.pic_gauss_residual(None, None, None, None, None, None) == L.PIC_E_ARG
    assert piclib.pic_beam_fields(None, None, None, None) == L.PIC_E_ARG
    assert piclib.pic_gather_push_deposit_multi(None, 2, None, None, None, None, None) == L.PIC_E_ARG
    piclib.pic_destroy(None)
