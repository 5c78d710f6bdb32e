"""No wide buffer store in the built library takes a register scalar offset.

A vector instruction that overwrites the data registers of a store of more
than 8 bytes right after it needs a wait state.  The compiler inserts it
when the store's scalar offset is a constant (and for global stores), but
not when it is a register, and on gfx950 such stores then sometimes wrote
the overwritten value (GEMM epilogue, first dword of 16-byte stores).  The
epilogue therefore keeps every offset of its 16-byte stores in the vector
register; this test reads the gfx950 assembly of the library as built and
checks that every buffer_store_dwordx3 / dwordx4 has a constant scalar
offset.  Host-only: it disassembles our own build.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_2309_00628_amd", "libmm.so")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"

WIDE_STORE = re.compile(r"\bbuffer_store_dwordx[34]\s+v\[\d+:\d+\],\s*(v\d+|off),\s*s\[\d+:\d+\],\s*(\S+)")


def test_wide_buffer_stores_use_a_constant_scalar_offset(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("libmm.so is not built")
    if not os.path.exists(OBJDUMP):
        pytest.skip("llvm-objdump not found")
    lib = tmp_path / "libmm.so"
    shutil.copy(LIB, lib)
    # extracts the bundled code objects next to the copy
    subprocess.run([OBJDUMP, "--offloading", str(lib)], cwd=tmp_path, check=True, capture_output=True)
    objs = sorted(p for p in tmp_path.iterdir() if p.name.endswith("gfx950"))
    assert objs, "no gfx950 code objects in the library"
    wide, bad = 0, []
    for obj in objs:
        asm = subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", str(obj)], check=True, capture_output=True,
                             text=True).stdout
        for line in asm.splitlines():
            m = WIDE_STORE.search(line)
            if not m:
                continue
            wide += 1
            soffset = m.group(2)
            if not re.fullmatch(r"-?(0x[0-9a-fA-F]+|\d+)", soffset):
                bad.append(f"{obj.name}: {line.strip()}")
    assert not bad, f"{len(bad)} of {wide} wide buffer stores use a register scalar offset:\n" + "\n".join(bad[:10])
