"""The Python binding's ctypes structures against the C header, and the
oracle's against its own C source: every field at the offset and with the size
the C compiler gives it, and every structure of the same size, so a field added
on one side only fails here, on the CPU."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# binding class -> C type
PAIRS = {"MeshDesc": "vls_mesh_desc", "SceneStats": "vls_scene_stats", "VoxelDesc": "vls_voxel_desc",
         "InstanceDesc": "vls_instance_desc", "ScannerDesc": "vls_scanner_desc", "PulseBatch": "vls_pulse_batch",
         "Outputs": "vls_outputs", "LaunchConfig": "vls_launch_config", "SurveyDesc": "vls_survey_desc",
         "Profile": "vls_profile", "TuneResult": "vls_tune_result"}


def _binding():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_vls_binding", os.path.join(ROOT, "paper_2101_09154_amd", "vls.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def c_layout():
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    vp = _binding()
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "vls.h"', "int main(void) {"]
    for py, c in PAIRS.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (py, c))
        for name, *_ in getattr(vp, py)._fields_:
            lines.append('printf("%s %s %%zu %%zu\\n", offsetof(%s, %s), sizeof(((%s*)0)->%s));'
                         % (py, name, c, name, c, name))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        r = subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr       # a binding field the header lacks fails to compile
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        parts = line.split()
        got[(parts[0], parts[1])] = tuple(int(x) for x in parts[2:])
    return vp, got


@pytest.mark.parametrize("py", sorted(PAIRS))
def test_binding_matches_header(c_layout, py):
    vp, got = c_layout
    cls = getattr(vp, py)
    assert ctypes.sizeof(cls) == got[(py, "sizeof")][0], py
    for name, *_ in cls._fields_:
        f = getattr(cls, name)
        assert (f.offset, f.size) == got[(py, name)], (py, name)


ORACLE_PAIRS = {"OrcScanner": "orc_scanner", "OrcVoxels": "orc_voxels", "OrcSurvey": "orc_survey"}


def test_oracle_binding_matches_its_source(orc):
    # the oracle's own ctypes mirrors against its C structures (compiled from
    # the oracle's source into a probe that prints the layout)
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "vls_oracle.c"', "int main(void) {"]
    for py, c in ORACLE_PAIRS.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (py, c))
        for name, *_ in getattr(orc, py)._fields_:
            lines.append('printf("%s %s %%zu %%zu\\n", offsetof(%s, %s), sizeof(((%s*)0)->%s));'
                         % (py, name, c, name, c, name))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        r = subprocess.run([cc, "-std=gnu11", "-fopenmp", "-I", os.path.join(ROOT, "oracle"), src, "-o", exe, "-lm"],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        parts = line.split()
        got[(parts[0], parts[1])] = tuple(int(x) for x in parts[2:])
    for py in ORACLE_PAIRS:
        cls = getattr(orc, py)
        assert ctypes.sizeof(cls) == got[(py, "sizeof")][0], py
        for name, *_ in cls._fields_:
            f = getattr(cls, name)
            assert (f.offset, f.size) == got[(py, name)], (py, name)
