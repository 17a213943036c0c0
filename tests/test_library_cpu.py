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
               "rtc_instance_info": rtc.InstanceInfoC, "rtc_telemetry_info": rtc.TelemetryInfoC,
               "rtc_pacer_stream": rtc.PacerStreamC, "rtc_pacer_desc": rtc.PacerDescC,
               "rtc_pacer_sample": rtc.PacerSampleC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rtc.h"', '#include "rtc_pacer.h"',
             "int main(void){"]
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


def test_mailbox_copy_check_rejects_torn_copies(tmp_path):
    """The waiter's check after copying a mailbox slot (a seqlock on the
    host's count of started frames): a writer thread that starts frame n,
    rewrites slot n % depth value by value and then publishes it races a
    reader that copies the slot of an already-published frame; every copy the
    check accepts must be whole (all values from that frame), and copies are
    accepted often."""
    import shutil
    import subprocess
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    src = tmp_path / "seq.cpp"
    src.write_text(r'''
#include <atomic>
#include <cstdio>
#include <mutex>
#include <thread>
#include <vector>
#include "rtc_seq.h"
int main() {
    const uint64_t depth = 3, n_act = 512, n_frames = 60000;
    std::vector<std::atomic<uint64_t>> mail(depth * n_act);
    for (auto &m : mail) m.store(~0ull);
    std::mutex mu;
    uint64_t seq = 0;                       // frames started (under mu)
    std::atomic<uint64_t> pub{0};           // frames published
    std::thread writer([&] {
        for (uint64_t n = 0; n < n_frames; ++n) {
            while (n - pub.load(std::memory_order_acquire) >= depth) {}
            { std::lock_guard<std::mutex> lk(mu); seq = n + 1; }
            for (uint64_t i = 0; i < n_act; ++i)
                mail[(n % depth) * n_act + i].store(n, std::memory_order_relaxed);
            pub.store(n + 1, std::memory_order_release);
        }
    });
    uint64_t accepted = 0, rejected = 0, torn = 0;
    std::vector<uint64_t> copy(n_act);
    for (;;) {
        const uint64_t p = pub.load(std::memory_order_acquire);
        if (p >= n_frames) break;
        if (p == 0) continue;
        const uint64_t q = p - 1;
        for (uint64_t i = 0; i < n_act; ++i)
            copy[i] = mail[(q % depth) * n_act + i].load(std::memory_order_relaxed);
        std::atomic_thread_fence(std::memory_order_acquire);
        uint64_t s;
        { std::lock_guard<std::mutex> lk(mu); s = seq; }
        if (!rtc::mailbox_copy_whole(s, q, depth)) { ++rejected; continue; }
        ++accepted;
        for (uint64_t i = 0; i < n_act; ++i) torn += copy[i] != q;
    }
    writer.join();
    std::printf("%llu %llu %llu\n", (unsigned long long)accepted, (unsigned long long)rejected,
                (unsigned long long)torn);
    return 0;
}
''')
    exe = tmp_path / "seq"
    csrc = os.path.join(ROOT, "paper_1903_01852_amd", "csrc")
    subprocess.run([cxx, "-O2", "-std=c++17", f"-I{csrc}", str(src), "-o", str(exe), "-lpthread"],
                   check=True)
    accepted, rejected, torn = map(int, subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True, timeout=120).stdout.split())
    assert torn == 0
    assert accepted > 100


def test_tile_flags_mark_a_frame_out_only_when_every_tile_is(tmp_path):
    """The waiter's readiness test on the per-tile flags: fixed cases (a flag
    short of the frame stops the scan, a tile already on a later frame counts,
    the scan resumes where it stopped), then writer threads that each own some
    tiles and, frame by frame in order, store a tile's value and then raise its
    flag (release) in a shuffled tile order, against a reader that waits for
    each frame with the scan (acquire loads) and checks every tile's value."""
    import shutil
    import subprocess
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    src = tmp_path / "flags.cpp"
    src.write_text(r'''
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>
#include "rtc_seq.h"
int main() {
    int bad = 0;
    {
        const uint64_t f[5] = {5, 5, 5, 4, 7};
        auto at = [&](int t) { return f[t]; };
        bad += rtc::tiles_ready_from(at, 5, 4, 0) != 3;     // tile 3 still on frame 3
        bad += rtc::tiles_ready_from(at, 5, 3, 0) != 5;     // every tile past frame 3
        bad += rtc::tiles_ready_from(at, 5, 4, 4) != 5;     // resumed after tile 3
        bad += rtc::tiles_ready_from(at, 0, 9, 0) != 0;     // no tiles: out
    }
    const int n = 96, n_writers = 4;
    const uint64_t n_frames = 20000;
    std::vector<std::atomic<uint64_t>> flag(n), val(n);
    for (int t = 0; t < n; ++t) { flag[t].store(0); val[t].store(~0ull); }
    std::vector<std::thread> writers;
    for (int w = 0; w < n_writers; ++w)
        writers.emplace_back([&, w] {
            std::mt19937 rng(w);
            std::vector<int> mine;
            for (int t = w; t < n; t += n_writers) mine.push_back(t);
            for (uint64_t q = 0; q < n_frames; ++q) {
                std::shuffle(mine.begin(), mine.end(), rng);
                for (int t : mine) {
                    val[t].store(q, std::memory_order_relaxed);
                    flag[t].store(q + 1, std::memory_order_release);
                }
            }
        });
    uint64_t torn = 0;
    for (uint64_t q = 0; q < n_frames; q += 7) {
        int tk = 0;
        while (tk < n)
            tk = rtc::tiles_ready_from(
                [&](int t) { return flag[t].load(std::memory_order_acquire); }, n, q, tk);
        for (int t = 0; t < n; ++t) torn += val[t].load(std::memory_order_relaxed) < q;
    }
    for (auto &w : writers) w.join();
    std::printf("%d %llu\n", bad, (unsigned long long)torn);
    return 0;
}
''')
    exe = tmp_path / "flags"
    csrc = os.path.join(ROOT, "paper_1903_01852_amd", "csrc")
    subprocess.run([cxx, "-O2", "-std=c++17", f"-I{csrc}", str(src), "-o", str(exe), "-lpthread"],
                   check=True)
    bad, torn = map(int, subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True, timeout=120).stdout.split())
    assert bad == 0
    assert torn == 0
