"""The slope exchange of the persistent frames, checked in the gfx950 code the
library was built into (no GPU needed).

Within a launch the workgroups exchange slopes and barrier words with relaxed
device-scope atomics and no acquire or release fence: a release at device
scope would write back the whole L2 of the workgroup's XCD every frame.  The
exchange is ordered instead by these facts of the built code, which this test
pins in the headline kernel's instructions:

- the slopes and the barrier's release words are stored device-coherently
  (``sc1``), so they do not stay in the writer's XCD-local L2;
- every wavefront waits for all of its stores (``s_waitcnt vmcnt(0)``) after
  its last device-coherent store and before the barrier's arrival atomic, so
  a workgroup arrives only once its slopes are stored;
- the release is polled and the slope slices are read with device-coherent
  loads (``sc1``), so no reader is served a stale line from its own L2; they
  are issued only after the poll saw the release (a load waited for, then a
  sleep and a branch back).
"""
import os
import re
import shutil
import struct
import subprocess
import tempfile

import pytest

from paper_1805_07254_amd import rtc

LLVM = "/opt/rocm/llvm/bin"
KERNEL = "_ZN4rtck12_GLOBAL__N_113frames_kernelILi0ELi4ELi2ELi8ELi2ELi16ELb0ELb0ELb0EEEvNS_11PersistArgsEiiii"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


def _code_objects(fatbin: bytes):
    """The gfx950 code objects of every offload bundle in a .hip_fatbin section."""
    out, i = [], fatbin.find(MAGIC)
    while i >= 0:
        n = struct.unpack_from("<Q", fatbin, i + len(MAGIC))[0]
        p = i + len(MAGIC) + 8
        for _ in range(n):
            off, size, idl = struct.unpack_from("<QQQ", fatbin, p)
            p += 24
            target = fatbin[p:p + idl].decode()
            p += idl
            if "gfx950" in target:
                out.append(fatbin[i + off:i + off + size])
        i = fatbin.find(MAGIC, i + 1)
    return out


@pytest.fixture(scope="module")
def isa():
    lib = rtc.LIB_PATH
    objcopy, objdump, readelf = _tool("llvm-objcopy"), _tool("llvm-objdump"), _tool("llvm-readelf")
    if not os.path.exists(lib):
        pytest.skip("librtc.so is not built")
    if not (objcopy and objdump and readelf):
        pytest.skip("LLVM binary tools not found")
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fatbin")
        subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", lib, os.path.join(d, "lib.copy")],
                       check=True, capture_output=True)
        for k, co in enumerate(_code_objects(open(fat, "rb").read())):
            path = os.path.join(d, f"co{k}.o")
            open(path, "wb").write(co)
            syms = subprocess.run([readelf, "-s", path], check=True, capture_output=True, text=True).stdout
            if re.search(rf"\s{re.escape(KERNEL)}$", syms, flags=re.M):
                dis = subprocess.run([objdump, "-d", f"--disassemble-symbols={KERNEL}", path], check=True,
                                     capture_output=True, text=True).stdout
                lines = [re.sub(r"//.*", "", ln).strip() for ln in dis.splitlines()]
                return [ln for ln in lines if ln and not ln.endswith(":") and not ln.startswith("Disassembly")]
    pytest.fail(f"{KERNEL} not found in the library's gfx950 code objects")


def _coherent_store(ln):
    return ln.startswith("global_store") and re.search(r"\bsc1\b", ln) is not None


def test_every_device_coherent_store_completes_before_the_next_arrival(isa):
    atomics = [i for i, ln in enumerate(isa) if ln.startswith("global_atomic_add")]
    assert len(atomics) >= 2, "no barrier arrival found"
    pending = None
    for i, ln in enumerate(isa):
        if _coherent_store(ln):
            pending = i
        elif ln.startswith("s_waitcnt") and "vmcnt(0)" in ln:
            pending = None
        elif ln.startswith("global_atomic_add"):
            assert pending is None, f"instruction {i} ({ln}) follows the coherent store {isa[pending]} unwaited"


def test_slopes_and_release_words_are_stored_device_coherently(isa):
    first_arrival = next(i for i, ln in enumerate(isa) if ln.startswith("global_atomic_add"))
    publishes = [ln for ln in isa[:first_arrival] if _coherent_store(ln) and ln.startswith("global_store_dword ")]
    assert len(publishes) >= 2, "slopes (x and y) not stored device-coherently before the first arrival"
    releases = [ln for ln in isa[first_arrival:] if _coherent_store(ln)]
    assert releases, "no device-coherent release store after the arrival"


def test_the_release_is_polled_with_device_coherent_loads(isa):
    polls = [i for i, ln in enumerate(isa) if ln.startswith("s_sleep")]
    assert polls, "no polling loop"
    for i in polls:
        # load, wait, compare and leave when released, count the spin, sleep, branch back
        window = isa[max(0, i - 12):i]
        assert any(ln.startswith("global_load_dword ") and re.search(r"\bsc1\b", ln) for ln in window), window
        assert any(ln.startswith("s_waitcnt") and "vmcnt(0)" in ln for ln in window), window
        assert isa[i + 1].startswith("s_branch"), isa[i:i + 2]


def test_slope_slices_are_read_with_device_coherent_loads(isa):
    # the wavefront's slices: 2 slices x 4 chunk groups x 4 elements, each a
    # 256-byte run of the exchange layout (element offsets 0, 256, 512, 768)
    loads = [ln for ln in isa if ln.startswith("global_load_dword ") and re.search(r"\bsc1\b", ln)]
    runs = [ln for ln in loads if re.search(r"offset:(256|512|768)\b", ln)]
    assert len(runs) >= 24, f"{len(runs)} device-coherent slice loads"
    plain = [ln for ln in isa if ln.startswith("global_load_dword ") and re.search(r"offset:(256|512|768)\b", ln)
             and not re.search(r"\bsc1\b", ln)]
    assert not plain, plain[:4]
