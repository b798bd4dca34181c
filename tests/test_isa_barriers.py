"""The HIP kernels compile for gfx950 with every barrier-carrying loop closed
by a lane-uniform back edge (see isa_barriers.py), without register spills in
the persistent worker, and with the default worker's machine code small
enough for the instruction cache (64 KiB, shared by two compute units): a
worker that outgrows it thrashes the cache and every phase slows down."""
import os
import re
import shutil
import subprocess

import pytest

from tests import isa_barriers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


MC = "/opt/rocm/llvm/bin/llvm-mc"
READELF = "/opt/rocm/llvm/bin/llvm-readelf"


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if shutil.which("/opt/rocm/bin/hipcc") is None:
        pytest.skip("hipcc not installed")
    from paper_1403_2056_amd import build
    out = tmp_path_factory.mktemp("isa") / "ssort.s"
    cmd = [build.HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", build.INCLUDE, "-I", build.CSRC, "-S", "--cuda-device-only", "-o", str(out),
           os.path.join(build.CSRC, "ssort_api.hip")]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return out


def test_no_barrier_in_lane_divergent_loop(asm):
    lines = asm.read_text().splitlines()
    kernels = list(isa_barriers.kernels(lines))
    assert len(kernels) >= 10
    bad = {k: b for k, body in kernels if (b := isa_barriers.check(body))}
    assert not bad, bad
    names = " ".join(k for k, _ in kernels)
    assert "k_worker" in names


def test_worker_without_spills(asm):
    text = asm.read_text()
    blocks = re.findall(r"\.name:\s+(\S+)\n(?:.*\n){0,40}?\s+\.private_segment_fixed_size:\s+(\d+)", text)
    workers = {n: int(sz) for n, sz in blocks if "k_worker" in n}
    assert len(workers) == 8, workers   # K in {4, 8} x chunk in {512, 1024} x byte or packed keys
    assert all(sz == 0 for sz in workers.values()), workers


@pytest.mark.skipif(not (os.path.exists(MC) and os.path.exists(READELF)), reason="llvm-mc not installed")
def test_worker_code_fits_instruction_cache(asm, tmp_path):
    obj = tmp_path / "ssort.o"
    subprocess.check_call([MC, "-triple=amdgcn-amd-amdhsa", "-mcpu=gfx950", "-filetype=obj", str(asm), "-o", str(obj)],
                          stderr=subprocess.DEVNULL)
    syms = subprocess.run([READELF, "-s", "--wide", str(obj)], capture_output=True, text=True, check=True).stdout
    size = {}
    for ln in syms.splitlines():
        f = ln.split()
        if len(f) >= 8 and f[3] == "FUNC" and "k_worker" in f[7]:
            size[f[7]] = int(f[2])
    assert len(size) == 8, size
    # the default worker (K = 4, chunk 512) and its alphabet-compression twin
    for z in ("Lb0E", "Lb1E"):
        w = [v for k, v in size.items() if "ILi4ELi512E" + z in k]
        assert w and w[0] < 64 * 1024, size


def _waited_before_barrier(body):
    """Every L2 write-back (the agent-scope release) is followed by a wait for
    the vector memory counter before the next barrier of the same straight
    path: the stores that publish after the barrier come from every wave, so
    the write-back must have finished by then.  Returns the offending lines."""
    bad = []
    for i, ln in enumerate(body):
        if "buffer_wbl2" not in ln:
            continue
        waited = False
        for nx in body[i + 1:]:
            t = nx.strip()
            if t.startswith("s_waitcnt") and ("vmcnt(0)" in t or t == "s_waitcnt 0"):
                waited = True
            if t.startswith("s_barrier") or t.startswith("s_endpgm"):
                break
        if not waited:
            bad.append(i)
    return bad


def test_release_waits_for_writeback_before_barrier(asm):
    lines = asm.read_text().splitlines()
    kernels = [(k, body) for k, body in isa_barriers.kernels(lines) if "k_worker" in k]
    assert len(kernels) == 8
    for k, body in kernels:
        assert any("buffer_wbl2" in b for b in body), k
        assert not _waited_before_barrier(body), k


def test_release_check_detects_a_missing_wait():
    body = ["\tglobal_store_dword v1, v2, s[0:1]", "\tbuffer_wbl2 sc1", "\ts_barrier", "\tglobal_store_dwordx2 v3, v[4:5], off sc1"]
    assert _waited_before_barrier(body) == [1]
    body.insert(2, "\ts_waitcnt vmcnt(0) expcnt(0) lgkmcnt(0)")
    assert _waited_before_barrier(body) == []


def test_no_flat_memory_access(asm):
    """Every load and store names its address space: a flat (generic) access
    also counts against the LDS wait counter, so each later LDS wait would
    wait for the global loads in flight (character gathers issued as flat
    loads serialised the kernels that interleave them with LDS work)."""
    lines = asm.read_text().splitlines()
    bad = {}
    for k, body in isa_barriers.kernels(lines):
        n = sum(1 for ln in body if ln.strip().startswith(("flat_load", "flat_store", "flat_atomic")))
        if n:
            bad[k] = n
    assert not bad, bad


def test_merge_without_scratch(asm):
    """The K-way merge's per-lane loser-tree build keeps its winners in
    registers (statically indexed), not in scratch memory."""
    text = asm.read_text()
    blocks = re.findall(r"\.name:\s+(\S+)\n(?:.*\n){0,40}?\s+\.private_segment_fixed_size:\s+(\d+)", text)
    merges = {n: int(sz) for n, sz in blocks if "k_mmerge" in n}
    assert len(merges) == 5, merges
    assert all(sz == 0 for sz in merges.values()), merges
