"""CPU emulation of the LDS-window simulation launches with 1024-thread
workgroups (no GPU needed).

emu/mkkernel.py copies sim_kernel's source for the host, and emu/emu_wg.cpp
runs it with one OS thread per GPU thread and several workgroups at once,
under AddressSanitizer. At the top of every step, all threads of a workgroup
must see the same frontier length, abort flag, step and simulation. Every
simulation's burnt cells, steps and trials must equal the oracle's on the
same Eq. 1 table, through the window launch (fires that reach a window edge
abort) and the whole-lattice re-run launch.

On the GPU, runs of this configuration stopped responding, and the planner
never gives a 1024-thread schedule a window. This test shows that the kernel's
logic at that size completes and is exact under the emulated semantics:
barriers, wave operations as rendezvous, and sequentially consistent memory.

The same small case also runs on 256-thread workgroups, the size of the
512x512 calibration schedule. The default cases run in about a minute.
FIRE_EMU_FULL=1 also runs the case
of the GPU failure: 512x512, a 128-cell window, 64 simulations and four
workgroups, about ten minutes.
"""
import os
import pathlib
import shutil
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1701_03549_amd import synth

EMU = pathlib.Path(__file__).resolve().parent / "emu"
REPO = pathlib.Path(__file__).resolve().parents[1]
BETA_STAR = (-3.0, -0.5, 6.0, 1.0, 2.0)
SEED = 0x5EED0001


def _compiler():
    # clang: the kernel source uses clang's vector types
    for cxx in ("/opt/rocm/llvm/bin/clang++", "clang++"):
        if shutil.which(cxx):
            return cxx
    pytest.skip("no clang++ for the host")


def _build(out, block):
    sys.path.insert(0, str(EMU))
    try:
        import mkkernel
    finally:
        sys.path.pop(0)
    mkkernel.generate(out / "kernel.inc")
    exe = out / f"emu_wg_{block}"
    cmd = [_compiler(), "-std=c++20", "-O1", "-g", "-fsanitize=address", "-pthread",
           f"-DEMU_BLOCK={block}", f"-I{out}", f"-I{EMU}", f"-I{REPO / 'include'}",
           str(EMU / "emu_wg.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.fixture(scope="module")
def emu_binary(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("emu_build"), 1024)


def _run_case(exe, tmp, W, H, land_seed, n, window, qcap, groups, global_bits=False):
    from paper_1701_03549_amd import fire
    ls = synth.make_landscape(W, H, land_seed)
    ign = synth.ignition_site(ls)
    ls["veg"].astype(np.uint8).tofile(tmp / "veg.bin")
    for key, name in (("elev_m", "elev"), ("slope_deg", "slope"), ("aspect_deg", "aspect"),
                      ("wind_to_deg", "wind")):
        np.ascontiguousarray(ls[key], dtype=np.float32).tofile(tmp / f"{name}.bin")
    T = oracle.thresholds(ls, BETA_STAR)
    np.ascontiguousarray(T, dtype=np.uint32).tofile(tmp / "table.bin")
    sims = fire.make_sims(n, 0, -1, ign)
    np.ascontiguousarray(sims).view(np.uint8).tofile(tmp / "sims.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    cmd = [str(exe), str(tmp), str(W), str(H), str(window), str(qcap), str(groups), hex(SEED)]
    r = subprocess.run(cmd + (["global"] if global_bits else []), capture_output=True, text=True,
                       env=env, timeout=3600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    got = np.fromfile(tmp / "emu_results.bin", np.uint8).view(fire.RESULT_DTYPE)
    reruns = int(r.stdout.split("re-runs ")[1].split(" ")[0])
    for i in range(n):
        o = oracle.simulate(ls["veg"], T, ign, int(sims[i]["sim_index"]), SEED, want_map=False)
        assert (int(got["burnt"][i]), int(got["steps"][i]), int(got["trials"][i])) == \
            (o["burnt"], o["steps"], o["trials"]), i
    return reruns


def test_window_1024_threads_small(emu_binary, tmp_path):
    """128x128 (landscape seed 6), 96-cell window, queues of 256 entries, 8
    simulations on two concurrent workgroups: two fires outgrow the window
    and are run again on the whole lattice, six do not."""
    reruns = _run_case(emu_binary, tmp_path, 128, 128, 6, 8, 96, 256, 2)
    assert 0 < reruns < 8


def test_window_256_threads_small(tmp_path):
    """The workgroup size of the 512x512 calibration schedule: the same case
    on 256-thread workgroups, four at once."""
    exe = _build(tmp_path, 256)
    reruns = _run_case(exe, tmp_path, 128, 128, 6, 8, 96, 256, 4)
    assert 0 < reruns < 8


def test_global_bitset_reruns_256_threads(tmp_path):
    """The re-run launch with each workgroup's whole-lattice bitset in global
    memory (the form for lattices whose bitset does not fit LDS): the window
    runs that abort are repeated that way, and every result equals the
    oracle's."""
    exe = _build(tmp_path, 256)
    reruns = _run_case(exe, tmp_path, 128, 128, 6, 8, 96, 256, 4, global_bits=True)
    assert 0 < reruns < 8


@pytest.mark.skipif(os.environ.get("FIRE_EMU_FULL") != "1", reason="about ten minutes; FIRE_EMU_FULL=1")
def test_window_1024_threads_gpu_failure_case(emu_binary, tmp_path):
    """512x512 (landscape seed 102), 128-cell window, queues of 1024 entries,
    64 simulations at the calibration vector, four concurrent workgroups."""
    reruns = _run_case(emu_binary, tmp_path, 512, 512, 102, 64, 128, 1024, 4)
    assert reruns > 0
