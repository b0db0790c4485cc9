"""Identity of a built kernel's machine code, for tying stored counter figures to the code they
were taken on.

A counter summary (HBM bytes of one launch) holds only for the machine code that was measured.
Hashing the source is too coarse: an edit to one template instantiation changes the file but
leaves the others' code as it was.  ``kernel_code_digest`` hashes the gfx950 instructions of one
kernel of the in-tree library and of every function it calls (transitively), with the two
position-dependent operands normalised: the PC-relative offset of a call (replaced by the callee's
name) or of a data reference, and the addresses in the disassembler's comments.  Two builds that
give the kernel the same instructions give the same digest, wherever the linker placed it.

Reads the library this repository builds (the offload bundle embedded in libhfx.so) with the ROCm
disassembler; returns None when that tool is missing.
"""
from __future__ import annotations

import hashlib
import os
import re
import shutil
import struct
import subprocess
import tempfile

from .build import LIB

_BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _objdump():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    p = os.path.join(rocm, "llvm", "bin", "llvm-objdump")
    return p if os.path.exists(p) else shutil.which("llvm-objdump")


def code_objects(lib: str = LIB, arch: str = "gfx950"):
    """The device code objects for ``arch`` in the library's uncompressed offload bundles."""
    with open(lib, "rb") as f:
        d = f.read()
    out, i = [], 0
    while (i := d.find(_BUNDLE_MAGIC, i)) >= 0:
        n = struct.unpack_from("<Q", d, i + 24)[0]
        p = i + 32
        for _ in range(n):
            off, size, tl = struct.unpack_from("<QQQ", d, p)
            p += 24
            triple = d[p:p + tl].decode()
            p += tl
            if triple.endswith("--" + arch):
                out.append(d[i + off:i + off + size])
        i += len(_BUNDLE_MAGIC)
    return out


def _functions(co: bytes, objdump: str):
    """{symbol: [(address, instruction text)]} and {address: symbol} of one code object."""
    with tempfile.NamedTemporaryFile(suffix=".co") as f:
        f.write(co)
        f.flush()
        txt = subprocess.run([objdump, "-d", "--no-show-raw-insn", f.name], capture_output=True, text=True,
                             check=True).stdout
    funcs, at, cur = {}, {}, None
    for line in txt.splitlines():
        m = re.match(r"^([0-9a-f]+) <(\S+)>:$", line)
        if m:
            cur = m.group(2)
            funcs[cur] = []
            at[int(m.group(1), 16)] = cur
            continue
        m = re.match(r"^\s+(\S.*?)\s*//\s*([0-9A-Fa-f]+):", line)
        if m and cur is not None:
            funcs[cur].append((int(m.group(2), 16), m.group(1)))
    return funcs, at


def _last_operand(ins: str) -> int:
    return int(ins.split(",")[-1].strip(), 0) & 0xFFFFFFFF


def kernel_code_digest(kernel: str, lib: str = LIB):
    """sha256 of ``kernel``'s instructions and those of the functions it calls; None if the
    disassembler is missing.  Raises KeyError if no code object holds ``kernel``."""
    objdump = _objdump()
    if objdump is None:
        return None
    for co in code_objects(lib):
        funcs, at = _functions(co, objdump)
        if kernel in funcs:
            return digest_of(kernel, funcs, at)
    raise KeyError(kernel)


def digest_of(kernel: str, funcs, at):
    """The digest over a disassembly: ``funcs`` maps a symbol to its [(address, instruction)],
    ``at`` an address to the symbol that starts there."""
    h, seen, todo = hashlib.sha256(), set(), [kernel]
    while todo:
        name = todo.pop(0)
        if name in seen:
            continue
        seen.add(name)
        ins, norm, k = funcs[name], [], 0
        while k < len(ins):
            a, t = ins[k]
            # s_getpc_b64 then a 64-bit add of a literal: a PC-relative address (a call target or data)
            if (t.startswith("s_getpc_b64") and k + 2 < len(ins) and ins[k + 1][1].startswith("s_add_u32")
                    and ins[k + 2][1].startswith("s_addc_u32")):
                off = (_last_operand(ins[k + 2][1]) << 32) | _last_operand(ins[k + 1][1])
                if off >= 1 << 63:
                    off -= 1 << 64
                target = at.get(a + 4 + off, "data")
                if target != "data":
                    todo.append(target)
                norm += [t, re.sub(r",[^,]*$", f", <{target}>", ins[k + 1][1]),
                         re.sub(r",[^,]*$", ", <hi>", ins[k + 2][1])]
                k += 3
                continue
            norm.append(t)
            k += 1
        h.update(f"{name}\n{len(norm)}\n".encode() + "\n".join(norm).encode() + b"\n")
    return h.hexdigest()


def k_main_symbol(tile_r: int, prec_kernel: int) -> str:
    """Mangled name of the main build kernel for a terms-3/4 output width and precision variant
    (0: FP64 only, 1: FP64 and FP32 tiers, 2: FP64, FP32 and split-BF16x3 tiers)."""
    return f"_ZN3hfx6k_mainILi{tile_r}ELi{prec_kernel}EEEvNS_7DevPlanENS_7KParamsE"
