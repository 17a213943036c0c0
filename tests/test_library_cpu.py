"""Host-side checks of the C ABI that need no GPU: exports, argument checks."""
import ctypes as C
import os
import re

import pytest

from paper_1903_01852_amd import rtc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(rtc_[a-z_0-9]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported():
    L = rtc.lib()
    declared = _declared()
    assert {"rtc_create", "rtc_load_matrices", "rtc_submit_pixel_chunk",
            "rtc_wait_commands"} <= declared
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(rtc.EXPORTS) == declared


def test_strerror_names_every_status():
    L = rtc.lib()
    for code in rtc.STATUS:
        assert L.rtc_strerror(code)
    assert L.rtc_strerror(0) == b"ok"


def test_null_and_bad_arguments_are_rejected_before_device_work():
    L = rtc.lib()
    assert L.rtc_create(None, None) == -1
    h = C.c_void_p()
    desc = rtc.CreateDescC(device=0, n_inst=0, inst=None, ring_depth=4, mode=0)
    assert L.rtc_create(C.byref(desc), C.byref(h)) == -1
    assert L.rtc_destroy(None) == -1
    assert L.rtc_get_info(None, 0, None) == -1
    assert L.rtc_submit_pixel_chunk(None, 0, 0, 0, 0, None) == -1
    assert L.rtc_wait_commands(None, 0, 0, None, 0, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the public structs have the C compiler's sizes and offsets."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"rtc_wfs_desc": rtc.WfsDescC, "rtc_instance_desc": rtc.InstanceDescC,
               "rtc_create_desc": rtc.CreateDescC, "rtc_frame_info": rtc.FrameInfoC,
               "rtc_instance_info": rtc.InstanceInfoC, "rtc_telemetry_info": rtc.TelemetryInfoC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rtc.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)
