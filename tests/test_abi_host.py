"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every entry point include/mcslam.h declares,
and agree with the binding on struct layouts.  Without a GPU, creating a
context must fail with a status code and a message, not abort.
"""

import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcslam.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_18056_amd import abi
    if not os.path.exists(abi.LIB_PATH):
        pytest.fail("libmcslam.so is not built (run __graft_entry__.build())")
    return abi.lib()


def test_exports_every_declared_entry_point(lib):
    names = declared_functions()
    assert {"mcs_init_map", "mcs_load_keyframes", "mcs_filter_step", "mcs_get_particles"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2504_18056_amd",
                                                                     "libmcslam.so")],
                         stdout=subprocess.PIPE, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mcs_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_version_and_error_strings(lib):
    from paper_2504_18056_amd import abi
    assert abi.mcs_version().startswith("mcslam")
    assert isinstance(abi.mcs_last_error(), str)


def test_struct_layouts_match_header():
    """Compile a C probe of sizeof/offsetof of every field against the header and
    compare with the ctypes structures of the binding."""
    import ctypes as C

    from paper_2504_18056_amd import abi
    structs = {"mcs_grid_desc": abi.GridDesc, "mcs_voxel_desc": abi.VoxelDesc,
               "mcs_step_params": abi.StepParams, "mcs_step_stats": abi.StepStats,
               "mcs_profile": abi.Profile, "mcs_request_times": abi.RequestTimes,
               "mcs_server_stats": abi.ServerStats}
    body = []
    for name, cls in structs.items():
        body.append('  printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            body.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    probe = "#include <stdio.h>\n#include <stddef.h>\n#include \"mcslam.h\"\nint main(void) {\n%s\n  return 0;\n}\n" % (
        "\n".join(body))
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(src, "w").write(probe)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        lines = subprocess.run([exe], stdout=subprocess.PIPE, text=True, check=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in lines if line)
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == int(got["%s.%s" % (name, field)]), (name, field)


def test_create_without_gpu_reports_an_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2504_18056_amd import abi
    with pytest.raises(abi.McsError) as e:
        abi.mcs_create(0)
    assert e.value.status in (abi.MCS_EDEVICE, abi.MCS_EINVAL)


def test_null_arguments_are_rejected(lib):
    import ctypes as C
    from paper_2504_18056_amd import abi
    assert lib.mcs_create(0, 0, None) == abi.MCS_EINVAL
    assert lib.mcs_memory_in_use(None, None) == abi.MCS_EINVAL
    assert lib.mcs_filter_step(None, 1, None, 1, None, None) == abi.MCS_EINVAL
    assert lib.mcs_get_particles(None, 1, None, None, None, None, None, None, None) == abi.MCS_EINVAL
    assert lib.mcs_destroy(None) == abi.MCS_OK
    assert lib.mcs_load_gicp_keyframes(None, 1, None, None, None) == abi.MCS_EINVAL
    assert lib.mcs_filter_step_gicp(None, 1, None, None, 1, None, None) == abi.MCS_EINVAL
    assert lib.mcs_filter_step_gicp_dev(None, 1, None, None, 1, None, None, None) == abi.MCS_EINVAL
    assert lib.mcs_get_gicp_system(None, 1, None, None) == abi.MCS_EINVAL
    assert lib.mcs_server_create(None, 0, 0, 0, 1, 0, None) == abi.MCS_EINVAL
    assert lib.mcs_server_drain(None) == abi.MCS_EINVAL
    assert lib.mcs_server_destroy(None) == abi.MCS_OK
    assert "NULL" in abi.mcs_last_error()
    del C


def test_plain_c_program_links_and_calls_the_library(lib):
    """A C99 program includes the header, links libmcslam.so and calls the
    entry points that need no device (version, errors, argument checks)."""
    from paper_2504_18056_amd import abi
    src = r'''
#include <stdio.h>
#include <string.h>
#include "mcslam.h"
int main(void) {
    mcs_ctx *ctx = NULL;
    int32_t map = 0;
    if (strncmp(mcs_version(), "mcslam", 6) != 0) return 1;
    if (mcs_init_map(NULL, NULL, NULL, &map) != MCS_EINVAL) return 2;
    if (strlen(mcs_last_error()) == 0) return 3;
    if (mcs_session_destroy(NULL, 1) != MCS_EINVAL) return 4;
    if (mcs_destroy(ctx) != MCS_OK) return 5;
    printf("ok\n");
    return 0;
}
'''
    libdir = os.path.dirname(abi.LIB_PATH)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        exe = os.path.join(d, "m")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), c,
                        "-L", libdir, "-lmcslam", "-Wl,-rpath," + libdir, "-o", exe], check=True)
        r = subprocess.run([exe], stdout=subprocess.PIPE, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.returncode


def test_outputs_are_sized_from_the_session(monkeypatch):
    """The getters allocate from mcs_session_info, never from caller sizes: a
    stale N, K or neighbour count is refused before the library writes."""
    import ctypes as C

    from paper_2504_18056_amd import abi

    calls = []

    class FakeLib:
        def mcs_session_info(self, ctx, sid, n, k, m, nb):
            for ref, v in ((n, 10), (k, 3), (m, 64), (nb, 4)):
                C.cast(ref, C.POINTER(C.c_int32))[0] = v
            return abi.MCS_OK

        def mcs_get_particles(self, ctx, sid, *ptrs):
            calls.append("particles")
            return abi.MCS_OK

        def mcs_get_neighbors(self, ctx, sid, out, k):
            calls.append("neighbors")
            C.cast(k, C.POINTER(C.c_int32))[0] = 4
            return abi.MCS_OK

        def mcs_last_error(self):
            return b"fake"

    monkeypatch.setattr(abi, "_lib", FakeLib())
    for bad in (dict(N=12), dict(N=10, K=5), dict(N=8)):
        with pytest.raises(abi.McsError) as e:
            abi.mcs_get_particles(None, 1, kf_poses=True, **bad)
        assert e.value.status == abi.MCS_EINVAL
    with pytest.raises(abi.McsError):
        abi.mcs_get_neighbors(None, 1, 10, 3)
    assert calls == []
    out = abi.mcs_get_particles(None, 1, kf_poses=True)
    assert out["poses"].shape == (10, 7) and out["kf_poses"].shape == (10, 3, 7)
    assert abi.mcs_get_neighbors(None, 1).shape == (10, 4)
    assert calls == ["particles", "neighbors"]
