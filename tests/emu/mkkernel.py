"""Writes a CPU-compilable copy of the simulation kernel's source.

Takes the part of csrc/fire_kernels.hip from the direction tables to the end
of sim_kernel, and the device structs of csrc/fire_internal.h, removes the
HIP qualifiers, maps LDS to the emulated workgroup's buffer, and inserts one
check at the top of sim_kernel's step loop (EMU_STEP_AGREE: every thread of
the workgroup sees the same frontier length, abort flag, step and
simulation). Nothing else of the kernel's text changes, so the emulation runs
the kernel's own control flow, indexing and synchronisation.
"""
import pathlib
import re
import sys

HERE = pathlib.Path(__file__).resolve().parent
CSRC = HERE.parents[1] / "paper_1701_03549_amd" / "csrc"


def generate(out_path):
    src = (CSRC / "fire_kernels.hip").read_text()
    internal = (CSRC / "fire_internal.h").read_text()
    body = src[src.index("// Geometry: direction d"):src.index("// LDS words of one wavefront of simw_kernel.")]
    structs = internal[internal.index("constexpr int kMaxDim"):internal.index("// Launchers (fire_kernels.hip)")]
    anchor = "aborted = WIN && ctl[kAbort0 + slot] != 0u;"
    if body.count(anchor) != 1:
        raise RuntimeError("step-loop anchor not found once in sim_kernel")
    body = body.replace(anchor, anchor + "\n      EMU_STEP_AGREE(n_cur, aborted, step, sim);")
    subs = [
        (r"__attribute__\(\(address_space\(1\)\)\)", ""),
        (r"extern __shared__ uint32_t lds\[\];", "uint32_t *lds = g_lds;"),
        (r"__launch_bounds__\(\w+\)", ""),
        (r"__global__", ""), (r"__device__", ""), (r"__constant__", ""), (r"__host__", ""),
        (r"__forceinline__", "inline"), (r"__restrict__", ""),
        (r"#pragma unroll( \d+)?", ""),
    ]
    for pat, rep in subs:
        body = re.sub(pat, rep, body)
        structs = re.sub(pat, rep, structs)
    text = "\n".join(['#include "hip_cpu.h"', '#include "fire.h"', "namespace firegpu {", structs,
                      body, "}  // namespace firegpu", ""])
    pathlib.Path(out_path).write_text(text)


if __name__ == "__main__":
    generate(sys.argv[1])
