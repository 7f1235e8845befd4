"""CPU-only checks of the C-ABI library: it builds, loads, exports every
symbol the public header declares, and its host-side paths behave without a
GPU (no compute is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bosmusic.h")


def _lib():
    import paper_1910_11872_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1910_11872_amd import build
        build.build()
    return pkg, pkg.lib()


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bosmusic_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("bosmusic_create", "bosmusic_destroy", "bosmusic_demodulate", "bosmusic_integrate"):
        assert name in fns


def test_library_exports_every_header_symbol():
    pkg, L = _lib()
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(pkg.ABI_FUNCTIONS) == set(header_functions())


def test_version_and_status_strings():
    pkg, L = _lib()
    assert pkg.bosmusic_version() == 1
    assert pkg.bosmusic_status_string(0) == "ok"
    assert pkg.bosmusic_status_string(-1) == "invalid argument"
    assert pkg.bosmusic_status_string(-2) == "unsupported"
    assert pkg.bosmusic_status_string(12345) == "unknown status"


def test_struct_layout_matches_compiled_header(tmp_path):
    """The ctypes structures have the sizes and offsets a C compiler gives the header."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pkg, _ = _lib()
    src = tmp_path / "layout.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"bosmusic.h\"\n"
        "#define F(T, m) printf(\"%s.%s %zu\\n\", #T, #m, offsetof(T, m));\n"
        "int main(void) {\n"
        "  printf(\"bosmusic_frame %zu\\n\", sizeof(bosmusic_frame));\n"
        "  printf(\"bosmusic_config %zu\\n\", sizeof(bosmusic_config));\n"
        "  printf(\"bosmusic_stats %zu\\n\", sizeof(bosmusic_stats));\n"
        "  printf(\"bosmusic_integrate_job %zu\\n\", sizeof(bosmusic_integrate_job));\n"
        + "".join(f"  F({t}, {m})\n" for t, cls in (("bosmusic_frame", pkg.bosmusic_frame),
                                                    ("bosmusic_config", pkg.bosmusic_config),
                                                    ("bosmusic_stats", pkg.bosmusic_stats),
                                                    ("bosmusic_integrate_job", pkg.bosmusic_integrate_job))
                  for m, _ in cls._fields_)
        + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for t, cls in (("bosmusic_frame", pkg.bosmusic_frame), ("bosmusic_config", pkg.bosmusic_config),
                   ("bosmusic_stats", pkg.bosmusic_stats), ("bosmusic_integrate_job", pkg.bosmusic_integrate_job)):
        assert int(got[t]) == ctypes.sizeof(cls), t
        for m, _ in cls._fields_:
            assert int(got[f"{t}.{m}"]) == getattr(cls, m).offset, (t, m)


def test_struct_layout_matches_header():
    pkg, _ = _lib()
    # bosmusic_frame: pointer, 3 x int32, int64, 2 x int32, uint32, 6 pointers
    assert ctypes.sizeof(pkg.bosmusic_frame) == 96
    assert pkg.bosmusic_frame.row_stride.offset == 24
    assert pkg.bosmusic_frame.omega_x.offset == 48
    assert ctypes.sizeof(pkg.bosmusic_config) == 32
    assert pkg.bosmusic_config.tune_cache.offset == 24
    assert ctypes.sizeof(pkg.bosmusic_stats) == 88


def test_null_arguments_are_rejected_without_device_work():
    pkg, L = _lib()
    assert L.bosmusic_create(None, None) == pkg.BM_E_INVALID_ARG
    assert L.bosmusic_demodulate(None, None, 0, 0, None) == pkg.BM_E_INVALID_ARG
    assert L.bosmusic_integrate(None, None, None, 1, 1, 1, 1, 0.0, 0.0, None, None) == pkg.BM_E_INVALID_ARG
    assert L.bosmusic_get_stats(None, None, 0, None) == pkg.BM_E_INVALID_ARG
    assert L.bosmusic_surrogate_get_state(None, None, 0, None) == pkg.BM_E_INVALID_ARG
    assert L.bosmusic_surrogate_set_state(None, None, 0, 0) == pkg.BM_E_INVALID_ARG
    assert L.bosmusic_destroy(None) == pkg.BM_OK
    cfg = pkg.bosmusic_config(0, 0, 64, 0, 0, None)
    h = ctypes.c_void_p()
    assert L.bosmusic_create(ctypes.byref(cfg), ctypes.byref(h)) == pkg.BM_E_INVALID_ARG
    assert h.value is None
    assert "max size" in pkg.bosmusic_last_error(None)


def test_create_without_gpu_reports_device_error():
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is visible")
    pkg, L = _lib()
    cfg = pkg.bosmusic_config(0, 64, 64, 0, 0, None)
    h = ctypes.c_void_p()
    assert L.bosmusic_create(ctypes.byref(cfg), ctypes.byref(h)) == pkg.BM_E_DEVICE
    assert h.value is None


def test_binding_has_no_cpu_fallback():
    """The package never imports the oracle and fails loudly without its library."""
    src = open(os.path.join(ROOT, "paper_1910_11872_amd", "__init__.py")).read()
    assert "oracle" not in src
    assert "raise ImportError" in src


def test_integrate_refuses_maps_not_row_major():
    """The binding checks layout before any library call: a transposed omega_y view
    (as numpy hands out for column-wise results) would otherwise be read in the wrong order."""
    import torch
    import paper_1910_11872_amd as pkg
    wx = torch.zeros(6, 5)
    wy_t = torch.zeros(5, 6).t()                     # shape (6, 5), column-major
    phi = torch.zeros(6, 5, dtype=torch.float64)
    with pytest.raises(ValueError):
        pkg.bosmusic_integrate(None, wx, wy_t, 2, 2, 0.0, 0.0, phi)
    with pytest.raises(ValueError):
        pkg.bosmusic_integrate_many(None, [(wx, wy_t, 2, 2, 0.0, 0.0, phi)])
    with pytest.raises(ValueError):
        pkg.bosmusic_integrate(None, wx, None, 2, 0, 0.0, 0.0, torch.zeros(6, 5))   # phi must be FP64


def test_frame_outputs_checked_for_dtype_shape_and_device():
    """The kernels store 4-byte omega/phase values and flag bytes into caller buffers:
    the binding refuses any other dtype (a float16 map would take out-of-bounds stores),
    shape or layout, and host tensors (the C ABI takes device pointers), before any
    library call."""
    import torch
    import paper_1910_11872_amd as pkg
    H, W = 6, 40
    fr = torch.zeros(H, W)
    ok32 = torch.zeros(H, W)
    bad = [dict(omega_x=torch.zeros(H, W, dtype=torch.float16)),
           dict(omega_x=torch.zeros(H, W, dtype=torch.bfloat16)),
           dict(omega_x=torch.zeros(H, W, dtype=torch.float64)),
           dict(omega_y=torch.zeros(W, H).t()),
           dict(omega_y=torch.zeros(H, W + 1)),
           dict(flags=torch.zeros(H, W, dtype=torch.int32)),
           dict(phase=torch.zeros(H, W, dtype=torch.float16))]
    for kw in bad:
        spec = pkg.FrameSpec(fr, 4, 16, pkg.BM_DIR_X | pkg.BM_DIR_Y, **{"omega_x": ok32, "omega_y": ok32, **kw})
        with pytest.raises(ValueError):
            pkg._marshal(spec)
    # correct dtypes and shapes, but host memory: refused as well
    spec = pkg.FrameSpec(fr, 4, 16, pkg.BM_DIR_X, omega_x=ok32, flags=torch.zeros(H, W, dtype=torch.uint8))
    with pytest.raises(ValueError, match="GPU"):
        pkg._marshal(spec)
    with pytest.raises(ValueError, match="GPU"):
        pkg.bosmusic_integrate(None, ok32, None, 2, 0, 0.0, 0.0, torch.zeros(H, W, dtype=torch.float64))


def test_surrogate_buffers_checked():
    import torch
    import paper_1910_11872_amd as pkg
    X = torch.zeros(64, 32)
    with pytest.raises(ValueError):
        pkg.bosmusic_surrogate_forward(None, X, torch.zeros(64, 2, dtype=torch.float16))
    with pytest.raises(ValueError):
        pkg.bosmusic_surrogate_forward(None, X, torch.zeros(64, 3))
    with pytest.raises(ValueError):
        pkg.bosmusic_surrogate_grad(None, X, torch.zeros(64, 2), torch.zeros(100))
    with pytest.raises(ValueError, match="GPU"):
        pkg.bosmusic_surrogate_forward(None, X, torch.zeros(64, 2))
