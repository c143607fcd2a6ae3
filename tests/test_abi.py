"""The C ABI library without a GPU: it loads, exports every function include/teno.h declares, the
Python binding covers exactly that set, and the host-only entry points behave (default options,
status strings, argument validation that returns before any HIP call)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "teno.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)       # drop comments
    text = re.sub(r"//[^\n]*", " ", text)
    names = set(re.findall(r"\b(teno_[a-z0-9_]+)\s*\(", text))
    assert len(names) > 20
    return names


@pytest.fixture(scope="module")
def T():
    from paper_1808_00037_amd import teno
    if not os.path.exists(teno.LIB_PATH):
        pytest.skip("libteno.so is not built")
    return teno


def test_every_declared_function_is_exported(T):
    declared = _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = declared - exported
    assert not missing, sorted(missing)
    L = ctypes.CDLL(T.LIB_PATH)
    for name in declared:
        assert getattr(L, name) is not None


def test_binding_covers_the_header(T):
    assert set(T._SIGS) == _declared()


def test_default_opts_are_the_papers_parameters(T):
    o = T.Opts()
    T.lib().teno_default_opts(ctypes.byref(o))
    assert o.scheme == T.TENO7X and o.alpha_mode == 0 and o.eps_mode == 0
    assert o.gamma == 1.4 and o.ct == 1e-5 and o.cfl == 0.5 and o.adv_speed == 1.0
    assert o.C == 1.0 and o.q == 6 and o.characteristic == 1


def test_status_strings(T):
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = T.lib().teno_status_str(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert T.lib().teno_status_str(-99)


def _grid(T, **kw):
    g = T.Grid(sys=T.EULER2D, nx=64, ny=32, bc_x=T.PERIODIC, bc_y=T.PERIODIC, dtype=T.F64,
               x0=0.0, x1=1.0, y0=0.0, y1=1.0)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=0), dict(sys=7), dict(sys=-1), dict(bc_x=2), dict(dtype=5),
                                 dict(x1=0.0), dict(y1=-1.0), dict(sys=1, ny=2), dict(nx=1 << 21),
                                 dict(nx=1 << 16, ny=1 << 16)])
def test_create_rejects_invalid_grids_before_touching_the_device(T, bad):
    o = T.Opts()
    T.lib().teno_default_opts(ctypes.byref(o))
    h = ctypes.c_void_p(123)
    code = T.lib().teno_create(ctypes.byref(_grid(T, **bad)), ctypes.byref(o), None, ctypes.byref(h))
    assert code == -1 and h.value is None


@pytest.mark.parametrize("field,value", [("gamma", 1.0), ("ct", 0.0), ("ct", 0.5), ("cfl", 0.0), ("scheme", 2),
                                         ("alpha_mode", 3), ("eps_mode", 2), ("q", 0), ("q", 13), ("C", 0.0),
                                         ("C", float("inf")), ("characteristic", 2)])
def test_create_rejects_invalid_options(T, field, value):
    o = T.Opts()
    T.lib().teno_default_opts(ctypes.byref(o))
    setattr(o, field, value)
    h = ctypes.c_void_p(123)
    code = T.lib().teno_create(ctypes.byref(_grid(T)), ctypes.byref(o), None, ctypes.byref(h))
    assert code == -1 and h.value is None


def test_null_arguments(T):
    L = T.lib()
    assert L.teno_create(None, None, None, None) == -1
    assert L.teno_destroy(None) == -1
    assert L.teno_rhs(None, None, None, None) == -1
    assert L.teno_run(None, None, 1, 0.0, 0, 0, None) == -1
    assert L.teno_batch_destroy(None) == -1
    assert L.teno_batch_set_shape(None, 4, 4, 1) == -1


@pytest.mark.parametrize("bad,code", [(dict(sys=0), -2), (dict(nx=0), -1), (dict(nx=1 << 21), -1),
                                      (dict(nx=40000, ny=20000), -1), (dict(sys=1, ny=3), -1),
                                      (dict(dtype=3), -1), (dict(x1=-1.0), -1)])
def test_batch_create_rejects_invalid_instances(T, bad, code):
    o = T.Opts()
    T.lib().teno_default_opts(ctypes.byref(o))
    grids = (T.Grid * 2)(_grid(T), _grid(T, **bad))
    h = ctypes.c_void_p(123)
    assert T.lib().teno_batch_create(grids, 2, ctypes.byref(o), None, ctypes.byref(h)) == code
    assert h.value is None


def test_batch_create_rejects_empty_and_null(T):
    o = T.Opts()
    T.lib().teno_default_opts(ctypes.byref(o))
    grids = (T.Grid * 1)(_grid(T))
    h = ctypes.c_void_p()
    assert T.lib().teno_batch_create(grids, 0, ctypes.byref(o), None, ctypes.byref(h)) == -1
    assert T.lib().teno_batch_create(None, 1, ctypes.byref(o), None, ctypes.byref(h)) == -1



def test_binding_rejects_host_buffers():
    # the C ABI takes plain device pointers: the binding refuses host tensors before any call
    import torch
    from paper_1808_00037_amd.teno import _WORD_TYPES, _buf
    for bad in (torch.zeros(10, dtype=torch.int32), None, "masks"):
        with pytest.raises(ValueError):
            _buf(bad, _WORD_TYPES, 10, "masks")


def test_workspace_bytes(T):
    """The device memory a context allocates by itself, as a function of the problem and of the
    reverse sweep's checkpoint interval (host arithmetic only)."""
    o = T.Opts()
    T.lib().teno_default_opts(ctypes.byref(o))
    L = T.lib()

    def ws(g, ck=0):
        return L.teno_workspace_bytes(ctypes.byref(g), ctypes.byref(o), ck)

    g2 = _grid(T, nx=4096, ny=4096)
    state = 4 * 4096 * 4096 * 8
    ctrl = ws(g2) - 3 * state                       # control block: the rest
    assert 0 < ctrl < 1 << 20
    assert ws(g2, 20) - ws(g2) == (3 * 20 + 5) * state
    g1 = _grid(T, sys=T.EULER1D, nx=4096, ny=1)
    assert ws(g1) == ctrl + 2 * 3 * 4096 * 8        # no y-part for one-dimensional systems
    g32 = _grid(T, dtype=T.F32)
    assert ws(g32) == ctrl + 3 * 4 * 64 * 32 * 4
    assert ws(_grid(T, nx=0)) == 0
    assert ws(g2, T.CKPT_STAGES) - ws(g2) == 4 * state     # every stage input stored: no segment scratch
    assert ws(g2, -2) == 0
    bad = T.Opts()
    T.lib().teno_default_opts(ctypes.byref(bad))
    bad.q = 0
    assert L.teno_workspace_bytes(ctypes.byref(g2), ctypes.byref(bad), 0) == 0
    assert T.workspace_bytes(T.EULER2D, 4096, 4096, ckpt_every=20) == ws(g2, 20)


def test_binding_constants_match_the_header():
    text = open(HEADER).read()
    m = re.search(r"#define\s+TENO_CKPT_STAGES\s+\((-?\d+)\)", text)
    assert m and int(m.group(1)) == -1
    from paper_1808_00037_amd import teno
    assert teno.CKPT_STAGES == int(m.group(1))
    m = re.search(r"#define\s+TENO_NOALLOC_SCRATCH_BYTES\s+\((\d+)u << (\d+)\)", text)
    assert m and teno.NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
