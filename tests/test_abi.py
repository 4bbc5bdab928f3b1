"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/bvh.h, and rejects invalid arguments with
the documented error codes before it touches a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bvh.h")


@pytest.fixture(scope="module")
def L():
    from paper_2511_15028_amd import bvh
    if not os.path.exists(bvh.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return bvh.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bvh_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("bvh_build", "bvh_trace", "bvh_trace_backward", "bvh_destroy", "bvh_get_stats",
              "bvh_read_buffer", "bvh_trace_counts", "bvh_last_error", "bvh_version",
              "bvh_closest_point", "bvh_closest_point_counts"):
        assert f in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_version(L):
    assert L.bvh_version() == 1


def test_build_argument_validation(L):
    from paper_2511_15028_amd import bvh
    h = ctypes.c_void_p(123)
    opts = bvh.BuildOpts(4, 0)
    fake = ctypes.c_void_p(0x1000)
    assert L.bvh_build(fake, 3, fake, 1, 0, ctypes.byref(opts), None, None) == bvh.EINVAL
    assert L.bvh_build(fake, 3, fake, -1, 0, ctypes.byref(opts), None, ctypes.byref(h)) == bvh.EINVAL
    assert h.value is None
    assert L.bvh_build(None, 3, fake, 1, 0, ctypes.byref(opts), None, ctypes.byref(h)) == bvh.EINVAL
    assert L.bvh_build(fake, 0, fake, 1, 0, ctypes.byref(opts), None, ctypes.byref(h)) == bvh.EINVAL
    assert L.bvh_build(fake, 3, fake, 1, 10, ctypes.byref(opts), None, ctypes.byref(h)) == bvh.EINVAL
    assert b"layout" in L.bvh_last_error()
    for bad in (bvh.BuildOpts(0, 5), bvh.BuildOpts(17, 0), bvh.BuildOpts(-1, 0),
                bvh.BuildOpts(4, 0, 0, 2)):
        assert L.bvh_build(fake, 3, fake, 1, 0, ctypes.byref(bad), None, ctypes.byref(h)) == bvh.EINVAL
    # the pbrt-q16 layout stores the triangle count in 4 bits
    sixteen = bvh.BuildOpts(16, 0)
    for lay in (bvh.LAYOUT_PBRT_Q16, bvh.LAYOUT_SG_EQ, bvh.LAYOUT_PBRT_Q16_SOAOS, bvh.LAYOUT_SG_EQ_A16):
        assert L.bvh_build(fake, 3, fake, 1, lay, ctypes.byref(sixteen), None,
                           ctypes.byref(h)) == bvh.EINVAL
        assert b"leaf_size" in L.bvh_last_error()
    res = bvh.BuildOpts(4, 0)
    res.reserved[2] = 1
    assert L.bvh_build(fake, 3, fake, 1, 0, ctypes.byref(res), None, ctypes.byref(h)) == bvh.EINVAL
    res = bvh.BuildOpts(4, 0, 12)
    assert L.bvh_build(fake, 3, fake, 1, 0, ctypes.byref(res), None, ctypes.byref(h)) == bvh.EINVAL
    assert L.bvh_build(fake, 3, fake, 1 << 27, 0, None, None, ctypes.byref(h)) == bvh.EUNSUPPORTED


def test_trace_and_backward_argument_validation(L):
    from paper_2511_15028_amd import bvh
    fake = ctypes.c_void_p(0x1000)
    assert L.bvh_trace(None, fake, 1, fake, 0, None) == bvh.EINVAL
    assert L.bvh_trace_counts(None, fake, 1, fake, 0, fake, None) == bvh.EINVAL
    assert L.bvh_trace_backward(fake, -1, fake, 1, fake, 1, fake, fake, fake, fake, None) == bvh.EINVAL
    assert L.bvh_trace_backward(fake, 3, fake, 1, None, 1, fake, fake, fake, fake, None) == bvh.EINVAL
    assert L.bvh_trace_backward(None, 0, None, 0, None, 0, None, None, None, None, None) == bvh.OK
    assert L.bvh_get_stats(None, None) == bvh.EINVAL
    assert L.bvh_read_buffer(None, 0, None, 0, None) == bvh.EINVAL
    assert L.bvh_closest_point(None, fake, 1, fake, None) == bvh.EINVAL
    assert L.bvh_closest_point(fake, fake, -1, fake, None) == bvh.EINVAL
    assert L.bvh_closest_point(fake, None, 1, fake, None) == bvh.EINVAL
    assert L.bvh_closest_point(fake, fake, 1 << 32, fake, None) == bvh.EUNSUPPORTED
    assert L.bvh_closest_point_counts(fake, fake, 1, fake, None, None) == bvh.EINVAL
    assert L.bvh_destroy(None) == bvh.OK


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors in bvh.py have the sizes and field offsets of the C
    structs in bvh.h (checked by compiling the header with gcc)."""
    import subprocess
    from paper_2511_15028_amd import bvh
    pairs = {"bvh_build_opts": bvh.BuildOpts, "bvh_stats": bvh.Stats,
             "bvh_scene_desc": bvh.SceneDesc, "bvh_tune_opts": bvh.TuneOpts,
             "bvh_batch_scene_info": bvh.SceneInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bvh.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('printf("bvh_ray %zu\\nbvh_hit %zu\\nbvh_tri %zu\\n", sizeof(bvh_ray), sizeof(bvh_hit), sizeof(bvh_tri));')
    lines.append('printf("bvh_point_query %zu\\nbvh_closest %zu\\n", sizeof(bvh_point_query), sizeof(bvh_closest));')
    lines.append("return 0; }")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c11", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True,
                                                               text=True, check=True).stdout.split("\n") if line)
    for cname, py in pairs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)
    assert (out["bvh_ray"], out["bvh_hit"], out["bvh_tri"]) == ("32", "16", "48")
    assert (out["bvh_point_query"], out["bvh_closest"]) == ("16", "16")


def test_batch_argument_validation(L):
    from paper_2511_15028_amd import bvh
    b = ctypes.c_void_p(7)
    descs = (bvh.SceneDesc * 2)()
    assert L.bvh_batch_create(descs, 0, None, None, ctypes.byref(b)) == bvh.EINVAL
    assert b.value is None
    descs[0].layout = 10
    assert L.bvh_batch_create(descs, 2, None, None, ctypes.byref(b)) == bvh.EINVAL
    descs[0].layout = bvh.LAYOUT_SHARED_SLAB  # carries boxes per stack entry: not batched
    assert L.bvh_batch_create(descs, 2, None, None, ctypes.byref(b)) == bvh.EUNSUPPORTED
    descs[0].layout = -1
    descs[1].stack_lds = 12
    assert L.bvh_batch_create(descs, 2, None, None, ctypes.byref(b)) == bvh.EINVAL
    descs[1].stack_lds = 0
    descs[1].n_tris = 5  # no mesh pointers
    assert L.bvh_batch_create(descs, 2, None, None, ctypes.byref(b)) == bvh.EINVAL
    assert L.bvh_batch_trace(None, None, None, None, None) == bvh.EINVAL
    assert L.bvh_batch_destroy(None) == bvh.OK
