"""The C-ABI library loads and exports every entry point include/dpcs.h declares (CPU only)."""
import ctypes
import os
import re
import subprocess

from paper_2503_12174_amd import dpcs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "dpcs.h")).read()
    return sorted(set(re.findall(r"DPCS_API\s+[\w\s\*]+?\b(dpcs_\w+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(dpcs.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = dpcs.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", dpcs.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (dpcs_\w+)", out))
    assert set(declared_symbols()) <= exported


def test_struct_layouts_match_the_header():
    """Sizes of the mirrored structs equal a C compiler's layout of the header's structs."""
    code = r'''
#include <stdio.h>
#include "dpcs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(dpcs_mesh_desc), sizeof(dpcs_scene_info), sizeof(dpcs_pinhole),
         sizeof(dpcs_render_params), sizeof(dpcs_render_aux), sizeof(dpcs_grads), sizeof(dpcs_request),
         sizeof(dpcs_profile), sizeof(dpcs_denoise_params), __builtin_offsetof(dpcs_render_params, seed));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "l")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(t) for t in (dpcs.MeshDesc, dpcs.SceneInfo, dpcs.Pinhole, dpcs.RenderParams,
                                       dpcs.RenderAux, dpcs.Grads, dpcs.Request, dpcs.Profile,
                                       dpcs.DenoiseParams)]
    want.append(dpcs.RenderParams.seed.offset)
    assert got == want


def test_calls_without_a_device_fail_cleanly():
    """No GPU here: creating a context reports an error instead of crashing."""
    import torch
    if torch.cuda.is_available():
        return
    h = ctypes.c_void_p()
    st = dpcs.lib().dpcs_context_create(0, None, 0, ctypes.byref(h))
    assert st != dpcs.OK and not h.value


def test_denoise_params_marshalling():
    """The binding's parameter block for the denoiser: one factor per guide channel, at
    most eight, and the default configuration matches the eight guide features."""
    import pytest
    from paper_2503_12174_amd import objective
    p = dpcs.denoise_params(640, 360, 3, 0.125, (1.0, 2.0, 3.0))
    assert (p.width, p.height, p.radius, p.guide_channels) == (640, 360, 3, 3)
    assert list(p.guide)[:3] == [1.0, 2.0, 3.0] and list(p.guide)[3:] == [0.0] * 5
    with pytest.raises(ValueError):
        dpcs.denoise_params(8, 8, 1, 0.1, [1.0] * 9)
    cfg = objective.DenoiseConfig()
    assert cfg.params(256, 256, 8).guide_channels == 8
    with pytest.raises(ValueError):
        cfg.params(256, 256, 7)
