"""The C ABI library loads and exports every entry point declared in
include/gdc.h (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gdc.h")
LIB = os.path.join(ROOT, "paper_2106_00449_amd", "libgdc.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(gdc_\w+)\s*\(", text, re.M)))


def test_header_declares_boundary():
    names = _declared()
    for required in ["gdc_init", "gdc_free", "gdc_last_error", "gdc_mobility_apply", "gdc_step",
                     "gdc_get_step", "gdc_set_step", "gdc_fluct_velocity", "gdc_predictor",
                     "gdc_philox_normals", "gdc_probe_kernel", "gdc_probe_read", "gdc_set_state",
                     "gdc_get_state", "gdc_batch_step", "gdc_step_log", "gdc_footprint", "gdc_device_bytes",
                     "gdc_get_launch_config", "gdc_set_launch_config"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first: python -m paper_2106_00449_amd.build"
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    lib.gdc_last_error.restype = ctypes.c_char_p
    assert lib.gdc_last_error() == b""


def test_init_rejects_null_config_without_touching_a_device():
    lib = ctypes.CDLL(LIB)
    h = ctypes.c_void_p()
    lib.gdc_last_error.restype = ctypes.c_char_p
    assert lib.gdc_init(None, ctypes.byref(h)) == -1
    assert b"cfg" in lib.gdc_last_error()
    assert lib.gdc_init(None, None) == -1
    lib.gdc_free(None)


def test_python_binding_marshals_config_layout():
    # the ctypes mirror of gdc_config must match the C struct layout
    import paper_2106_00449_amd as g
    c = g._Config
    assert c.L.offset == 0 and c.n.offset == 24
    assert ctypes.sizeof(g._Forces) == 8 * 12
    off = c.forces.offset
    assert off % 8 == 0 and c.device.offset == off + ctypes.sizeof(g._Forces)


def test_ctypes_layout_matches_c_compiler(tmp_path):
    import shutil
    import subprocess
    import paper_2106_00449_amd as g
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gdc.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(gdc_config), offsetof(gdc_config, seed), offsetof(gdc_config, shapes),'
                   'offsetof(gdc_config, forces), offsetof(gdc_config, device), offsetof(gdc_config, stream),'
                   'sizeof(gdc_stats), sizeof(gdc_shape));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    c = g._Config
    assert vals == [ctypes.sizeof(c), c.seed.offset, c.shapes.offset, c.forces.offset, c.device.offset,
                    c.stream.offset, ctypes.sizeof(g._Stats), ctypes.sizeof(g._Shape)]


def test_footprint_rejects_stencils_too_wide_for_averaging():
    # averaging keeps a blob's axis-2 factors in 64 entries: an envelope
    # spanning more than 58 grid points along axis 2 is refused at set-up
    # (gdc_footprint runs the same validation without a device)
    import pytest
    import paper_2106_00449_amd as g
    import workloads as wl
    w = wl.small_case("wide", n_bodies=4, n=(32, 32, 256), L=(24.0, 24.0, 24.0), precision="fp32")
    kw = wl.library_kwargs(w)
    g.footprint(**dict(kw, trunc=2.0))          # 2 trunc / dx + 1 = 43 points: accepted
    with pytest.raises(RuntimeError, match="at most 58"):
        g.footprint(**dict(kw, trunc=2.8))      # 60 points
