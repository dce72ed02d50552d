"""The C ABI on the CPU: the library loads, exports every symbol the header declares,
and validates arguments on the host before touching any device."""
import ctypes
import os
import re

import numpy as np
import pytest

from helpers import ROOT, ensure_built


@pytest.fixture(scope="module")
def lib():
    ensure_built()
    from paper_2503_01199_amd import _lib as L
    return L.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "gsr.h")).read()
    return re.findall(r"^\s*(?:gsr_status|void|const char \*|size_t)\s*(gsr_\w+)\s*\(", text, re.M)


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_2503_01199_amd import _lib as L
    assert set(header_functions()) == set(L.EXPORTS)


STRUCTS = {"GsrScene": "gsr_scene", "GsrCamera": "gsr_camera", "GsrOptions": "gsr_options",
           "GsrFrameInfo": "gsr_frame_info", "GsrFrameBuffers": "gsr_frame_buffers",
           "GsrAdamOptions": "gsr_adam_options", "GsrDensifyOptions": "gsr_densify_options"}


def test_struct_layouts_match_header_sizes(tmp_path):
    """The binding's ctypes structures have the sizes the C compiler gives the
    header's structures (compiled here with gcc against include/gsr.h)."""
    import subprocess
    from paper_2503_01199_amd import _lib as L
    src = tmp_path / "sizes.c"
    src.write_text("#include <stdio.h>\n#include \"gsr.h\"\nint main(void) {\n"
                   + "".join('  printf("%%s %%zu\\n", "%s", sizeof(%s));\n' % (c, c) for c in STRUCTS.values())
                   + "  return 0;\n}\n")
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    sizes = dict((a, int(b)) for a, b in (ln.split() for ln in subprocess.check_output([str(exe)], text=True).split("\n")
                                          if ln.strip()))
    for py, c in STRUCTS.items():
        assert ctypes.sizeof(getattr(L, py)) == sizes[c], (py, ctypes.sizeof(getattr(L, py)), sizes[c])


def _scene(n=10, deg=0):
    from paper_2503_01199_amd import _lib as L
    s = L.GsrScene()
    s.n = n
    s.sh_degree = deg
    dummy = 0x1000  # never dereferenced by the size query
    s.means = s.log_scales = s.quats = s.opacity_logits = s.sh = dummy
    return s


def _cams(V=1, W=64, H=48):
    from paper_2503_01199_amd import _lib as L
    cams = (L.GsrCamera * V)()
    for c in cams:
        c.width, c.height, c.fx, c.fy, c.cx, c.cy = W, H, 50.0, 50.0, W / 2, H / 2
        for k in range(3):
            c.R[4 * k] = 1.0
        c.near_plane = 0.2
    return cams


def _size(lib, scene, cams, V, opts, m=1000):
    from paper_2503_01199_amd import _lib as L
    out = ctypes.c_size_t(0)
    st = lib.gsr_workspace_size(None, ctypes.byref(scene), cams, V, ctypes.byref(opts), m, ctypes.byref(out))
    return st, out.value


def test_workspace_size_and_validation_on_host(lib):
    from paper_2503_01199_amd import _lib as L
    o = L.GsrOptions()
    st, b0 = _size(lib, _scene(1000), _cams(), 1, o, 0)
    assert st == L.GSR_OK and b0 > 0
    st, b1 = _size(lib, _scene(1000), _cams(), 1, o, 10_000)
    assert st == L.GSR_OK and b1 >= b0 + 16 * 10_000
    st, b2 = _size(lib, _scene(0), _cams(), 1, o, 0)
    assert st == L.GSR_OK  # an empty scene is valid
    bad = [
        (_scene(-1), _cams(), 1, o),
        (_scene(10, deg=4), _cams(), 1, o),
        (_scene(10), _cams(), 0, o),
        (_scene(10), _cams(V=65), 65, o),
        (_scene(10), _cams(W=0), 1, o),
    ]
    for sc, cams, V, opts in bad:
        assert _size(lib, sc, cams, V, opts)[0] == L.GSR_ERR_INVALID_ARG
    c = _cams()
    c[0].fx = -1.0
    assert _size(lib, _scene(), c, 1, o)[0] == L.GSR_ERR_INVALID_ARG
    c = _cams()
    c[0].near_plane = 0.0
    assert _size(lib, _scene(), c, 1, o)[0] == L.GSR_ERR_INVALID_ARG
    c = _cams()
    c[0].t[1] = float("nan")
    assert _size(lib, _scene(), c, 1, o)[0] == L.GSR_ERR_INVALID_ARG
    o2 = L.GsrOptions()
    o2.deterministic = 2
    assert _size(lib, _scene(), _cams(), 1, o2)[0] == L.GSR_ERR_INVALID_ARG
    o3 = L.GsrOptions()
    o3.precision = 7
    assert _size(lib, _scene(), _cams(), 1, o3)[0] == L.GSR_ERR_INVALID_ARG
    s = _scene()
    s.means = None
    assert _size(lib, s, _cams(), 1, o)[0] == L.GSR_ERR_INVALID_ARG


def test_null_context_is_rejected(lib):
    from paper_2503_01199_amd import _lib as L
    o = L.GsrOptions()
    imgs = (ctypes.c_void_p * 1)(0x1000)
    assert lib.gsr_forward(None, ctypes.byref(_scene()), _cams(), 1, ctypes.byref(o), 0x1000, 1 << 20, imgs,
                           None) == L.GSR_ERR_INVALID_ARG
    assert lib.gsr_variance(None, None, 0, None, None) == L.GSR_ERR_INVALID_ARG
    assert lib.gsr_sparse_adam(None, 0, 0, None, None, None, None, None, None, None) == L.GSR_ERR_INVALID_ARG
    assert lib.gsr_opacity_decay(None, None, 0, 0.5, None) == L.GSR_ERR_INVALID_ARG
    out = ctypes.c_size_t()
    assert lib.gsr_densify_workspace_size(None, 1000, 100, ctypes.byref(out)) == L.GSR_OK and out.value > 4000
    assert lib.gsr_densify_workspace_size(None, -1, 100, ctypes.byref(out)) == L.GSR_ERR_INVALID_ARG
    assert isinstance(lib.gsr_last_error(None), bytes)
    out = ctypes.c_size_t()
    assert lib.gsr_morton_workspace_size(None, 1000, ctypes.byref(out)) == L.GSR_OK and out.value > 8000


def test_context_without_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2503_01199_amd import _lib as L
    ctx = ctypes.c_void_p()
    assert lib.gsr_context_create(0, ctypes.byref(ctx)) == L.GSR_ERR_DEVICE


def test_python_binding_fails_loudly_without_library(tmp_path):
    from paper_2503_01199_amd import _lib as L
    with pytest.raises(RuntimeError, match="not built"):
        L.load(str(tmp_path / "libgsr.so"))


def test_scene_generators_are_deterministic():
    from paper_2503_01199_amd import scenes
    a = scenes.tiny_scene()
    b = scenes.tiny_scene()
    for x, y in zip(a.arrays(), b.arrays()):
        assert np.array_equal(x, y)
    assert a.means.dtype == np.float32 and a.sh.shape == (1024, 1, 3)
    s = scenes.spheres_planes_scene(5000)
    assert s.sh.shape == (5000, 16, 3) and np.isfinite(s.quats).all()
    assert np.allclose(np.linalg.norm(s.quats, axis=1), 1, atol=1e-5)
