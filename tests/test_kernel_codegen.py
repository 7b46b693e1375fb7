"""Code generation of the fold walk (CPU: hipcc cross-compiles gfx950 assembly).

The walk keeps two groups of 16-byte loads in flight per wave: while one group
is added, the next group's loads are outstanding.  That holds only if the
compiler's wait counting can wait for part of the outstanding loads
(`s_waitcnt vmcnt(k)`, k > 0); when it cannot tell the outstanding operations
apart (a pending store or a flat access reaching the walk) every wait becomes
`vmcnt(0)` and the walk serialises on each group (measured: 46 -> 49.4 us per
2^30-sample launch).  This checks every fold kernel's walk loop in the
assembly, and that the stream is read with global (not flat) loads.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2501_05993_amd", "csrc", "pcal_kernels.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("asm") / "pcal_kernels.s")
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "--cuda-device-only", "-S"]
    r = subprocess.run([HIPCC] + flags + [SRC, "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    funcs, cur = {}, None
    for line in open(out).read().split("\n"):
        m = re.match(r"^(_Z\w+):", line)
        if m:
            cur = m.group(1)
            funcs[cur] = []
        if cur:
            funcs[cur].append(line)
    return funcs


def _walk_loop(lines):
    """The longest loop with a workgroup barrier and at least 8 16-byte stream loads."""
    labels = {}
    for i, l in enumerate(lines):
        m = re.match(r"^(\.LBB\d+_\d+):", l)
        if m:
            labels[m.group(1)] = i
    best = None
    for i, l in enumerate(lines):
        m = re.search(r"s_c?branch\w*\s+(\.LBB\d+_\d+)", l)
        if not m or m.group(1) not in labels or labels[m.group(1)] >= i:
            continue
        body = lines[labels[m.group(1)]:i + 1]
        loads = sum("load_dwordx4" in x for x in body)
        if loads >= 8 and any("s_barrier" in x for x in body):
            if best is None or len(body) > len(best):
                best = body
    return best


def _fold_kernels(funcs):
    names = [n for n in funcs if "fold_kernel" in n or "fold_batch_kernel" in n]
    # {2,8}-bit x 3 precisions: plain, batched (device or inline work-list); plus the plain fixed-point form
    assert len(names) == 20, names
    return names


def test_walk_loops_wait_for_part_of_the_loads(asm):
    for name in _fold_kernels(asm):
        body = _walk_loop(asm[name])
        assert body is not None, "no walk loop found in " + name
        waits = [int(m.group(1)) for x in body for m in [re.search(r"s_waitcnt\s+vmcnt\((\d+)\)", x)] if m]
        assert waits, name
        assert max(waits) >= 5, "%s: walk waits %s (every load, no group in flight)" % (name, waits)


def test_walk_reads_the_stream_with_global_loads(asm):
    for name in _fold_kernels(asm):
        body = _walk_loop(asm[name])
        assert not any("flat_load" in x for x in body), name
        assert sum("global_load_dwordx4" in x and " nt" in x for x in body) >= 8, name
