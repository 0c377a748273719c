"""Checks of the gfx950 machine code in the built libpct.so (CPU only: the
device code objects are taken out of the library and disassembled with the
ROCm LLVM tools).

A kernel that reads a vector register which no instruction of the kernel
writes computes with garbage.  This happened once at -O2/-O3 with a slice
test variant that loaded four cells per lane as one 16-byte load: the loop
carried two lanes of the 128-bit ground vector through registers whose
copies the backend dropped, so the "ground differs from the slice below"
test read undefined values and every slice was kept on the GPU, while the
CPU build of the same source was right.  The scan below finds that class of
fault: per kernel, vector registers read but never written (v0-v2 hold the
work-item ids on entry and are excluded)."""
import os
import re
import shutil
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2403_07631_amd", "libpct.so")
LLVM = "/opt/rocm/llvm/bin"

# first operand is read, not written
_READ_ONLY = ("global_store", "buffer_store", "flat_store", "scratch_store", "ds_write", "ds_add_u32", "ds_add_f32",
              "ds_max", "ds_min", "ds_or", "ds_and", "ds_xor", "ds_inc", "ds_dec", "ds_sub")
_ATOMIC = ("global_atomic", "buffer_atomic", "flat_atomic")


def _regs(tok):
    out = set()
    for m in re.finditer(r"\bv\[(\d+):(\d+)\]|\bv(\d+)\b", tok):
        if m.group(3) is not None:
            out.add(int(m.group(3)))
        else:
            out.update(range(int(m.group(1)), int(m.group(2)) + 1))
    return out


def unwritten_vgprs(disasm):
    """{kernel: sorted VGPRs read but never written} from llvm-objdump text."""
    res, func = {}, None
    for line in disasm.splitlines():
        m = re.match(r"^[0-9a-f]+ <(\S+)>:", line)
        if m:
            func = m.group(1)
            res[func] = [set(), set()]
            continue
        if func is None:
            continue
        s = line.split("//")[0].strip()
        if not s or s.endswith(":"):
            continue
        parts = s.split(None, 1)
        if len(parts) < 2:
            continue
        op, args = parts
        ops = [a.strip() for a in args.split(",")]
        w, r = res[func]
        returns = op.startswith(_ATOMIC) and re.search(r"\b(sc0|glc)\b", args)
        if (op.startswith(_READ_ONLY) and "_rtn" not in op) or (op.startswith(_ATOMIC) and not returns):
            for a in ops:
                r |= _regs(a)
            continue
        w |= _regs(ops[0])
        if op.startswith(("v_mad_u64_u32", "v_mad_i64_i32")) and len(ops) >= 5:
            # a 32-bit multiply-add done by the 64-bit instruction leaves the
            # addend's high half undefined: only its low register is read
            m = re.match(r"v\[(\d+):\d+\]", ops[4])
            if m:
                ops = ops[:4] + [f"v{m.group(1)}"] + ops[5:]
        for a in ops[1:]:
            r |= _regs(a)
    return {f: sorted(r - w - {0, 1, 2}) for f, (w, r) in res.items() if r - w - {0, 1, 2}}


def code_objects(lib):
    """The gfx950 code objects of a HIP shared library's offload bundles."""
    tmp = lib + ".fatbin"
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", f".hip_fatbin={tmp}", lib, os.devnull],
                   check=True, capture_output=True)
    try:
        data = open(tmp, "rb").read()
    finally:
        os.remove(tmp)
    out = []
    for m in re.finditer(b"__CLANG_OFFLOAD_BUNDLE__", data):
        s = m.start()
        p = s + 24
        (cnt,) = struct.unpack_from("<Q", data, p)
        p += 8
        for _ in range(cnt):
            off, size, tl = struct.unpack_from("<QQQ", data, p)
            p += 24
            triple = data[p:p + tl].decode()
            p += tl
            if triple.endswith("gfx950"):
                out.append(data[s + off:s + off + size])
    return out


@pytest.mark.skipif(not (os.path.exists(LIB) and os.path.exists(os.path.join(LLVM, "llvm-objdump"))),
                    reason="needs the built library and the ROCm LLVM tools")
def test_kernels_write_every_register_they_read(tmp_path):
    cos = code_objects(LIB)
    assert len(cos) >= 5, "no gfx950 code objects found in libpct.so"
    bad, n_kernels = {}, 0
    for i, co in enumerate(cos):
        path = tmp_path / f"co{i}.o"
        path.write_bytes(co)
        dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", str(path)], check=True,
                             capture_output=True, text=True).stdout
        n_kernels += len(re.findall(r"^[0-9a-f]+ <\S+>:", dis, re.M))
        bad.update(unwritten_vgprs(dis))
    assert n_kernels > 50
    assert not bad, f"kernels read vector registers they never write: {bad}"


def test_scan_finds_a_dropped_copy():
    """The scan itself, on a hand-written listing: v7 is carried into a
    register that is then read without any write to it."""
    listing = """
0000000000001000 <k_demo>:
\tglobal_load_dwordx4 v[4:7], v[0:1], off                      // 000000001000: 00000000
\tv_cmp_neq_f32_e32 vcc, v51, v4                               // 000000001008: 00000000
\tv_mov_b32_e32 v8, v7                                         // 00000000100C: 00000000
\tglobal_store_dword v[0:1], v8, off                           // 000000001010: 00000000
\ts_endpgm                                                     // 000000001018: 00000000
"""
    assert unwritten_vgprs(listing) == {"k_demo": [51]}
    assert unwritten_vgprs(listing.replace("v51", "v8")) == {}
    # the high half of a 64-bit multiply-add's addend is not counted as read
    mad = listing.replace("v_mov_b32_e32 v8, v7", "v_mad_u64_u32 v[8:9], s[0:1], v4, s2, v[6:7]")
    mad = mad.replace("v51", "v4").replace("global_load_dwordx4 v[4:7]", "global_load_dwordx2 v[4:5]")
    assert unwritten_vgprs(mad) == {"k_demo": [6]}
