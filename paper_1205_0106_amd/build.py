"""Build libamqmc.so (HIP, gfx950) in-tree.

Steps: write the Sobol direction-number table (from SciPy's engine, checked
against its points), embed it with an assembler ``.incbin``, compile the HIP
translation units for gfx950 and link the shared library next to this
file.  Object files go to ``<repo>/_build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libamqmc.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 ops are disabled for all device code on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
SOURCES = ["amq_kernels.hip", "amq_engine.hip", "amq_sweep_f32_mono.hip", "amq_sweep_f32_lag.hip",
           "amq_sweep_f64_mono.hip", "amq_sweep_f64_lag.hip"]


def _table_object() -> str:
    os.makedirs(BUILD, exist_ok=True)
    binp = os.path.join(BUILD, "sobol_v32.bin")
    sys.path.insert(0, CSRC)
    try:
        import gen_sobol_table
    finally:
        sys.path.pop(0)
    dims = gen_sobol_table.main(binp)
    asm = os.path.join(BUILD, "amq_sobol_table.S")
    with open(asm, "w") as f:
        f.write(f"""    .section .rodata
    .p2align 6
    .globl amq_sobol_v32
    .type amq_sobol_v32, @object
amq_sobol_v32:
    .incbin "{binp}"
    .size amq_sobol_v32, . - amq_sobol_v32
    .p2align 2
    .globl amq_sobol_v32_dims
    .type amq_sobol_v32_dims, @object
amq_sobol_v32_dims:
    .long {dims}
    .size amq_sobol_v32_dims, 4
    .section .note.GNU-stack,"",@progbits
""")
    obj = os.path.join(BUILD, "amq_sobol_table.o")
    subprocess.run(["gcc", "-c", "-fPIC", asm, "-o", obj], check=True)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libamqmc.so."""
    os.makedirs(BUILD, exist_ok=True)
    objs = [_table_object()]
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines()
                 if "packed-fp32-ops" not in ln and ln.strip() and "warning generated" not in ln]
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and lines:
            print(text)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(f"--- {s}\n{t}" for s, t in failed))
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
