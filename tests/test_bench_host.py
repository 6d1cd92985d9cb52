"""Host-side logic of bench.py (no GPU): the command-line contract for more
than one GPU, the launches a stage runs, and the algorithmic work counts."""
import json
import os
import subprocess
import sys

import bench
from paper_2406_19494_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_step_kernels_of_each_family():
    # (2D/3D flux kernels compute the velocity derivatives themselves: no
    # derivative launch in a step)
    tgv, _ = W.tgv(8)
    assert bench.step_kernel_ids(tgv) == [0, 8, 7, 6]
    tgv_inviscid, _ = W.tgv(8, viscous=False)
    assert bench.step_kernel_ids(tgv_inviscid) == [0, 8, 7, 6]
    ch, _ = W.channel(16, 8, 8)
    assert bench.step_kernel_ids(ch) == [0, 8, 7, 6]  # body force, periodic z: fused
    ch.bc = ch.bc[:4] + ("wall", "wall")
    assert bench.step_kernel_ids(ch) == [0, 7, 3, 4]  # body force, walls in z: unfused
    bl, _, _ = W.porous_bl(nx=16, ny=8)
    assert bench.step_kernel_ids(bl) == [0, 8, 1, 6]
    sod, _ = W.sod(50)
    assert bench.step_kernel_ids(sod) == [0, 1, 4]


def test_algorithmic_counts():
    case, _ = W.tgv(8)
    nbox = 14 ** 3
    # halo fill: U read once (5 values per cell), 7 primitives written per box cell
    assert bench.algorithmic_bytes(case, "k_prim_halo") == 8 * (512 * 5 + nbox * 7)
    assert bench.algorithmic_bytes(case, "k_prim_ghost") == 8 * 2 * 7 * (nbox - 512)
    # update: 5 fluxes of every face of the 3 directions, Un and Uin read, Uout written
    faces = 3 * 9 * 8 * 8
    assert bench.algorithmic_bytes(case, "k_update") == 8 * (5 * faces + 3 * 512 * 5)
    # flux work per face: 10 reconstructions, HLLC, viscous terms (3D)
    assert bench.FLOPS_PER_FACE[(3, True)] == 10 * 69 + 79 + 183


def test_counter_summaries_parse_or_are_absent():
    # the committed summaries either match the kernel sources (numbers) or
    # are reported as missing (None), never a parse error
    for w in ("tgv64", "channel"):
        for k in ("k_flux_xy", "k_flux_update", "k_prim_halo"):
            t = bench.measured_traffic(k, w)
            v = bench.measured_valu(k, w)
            assert t is None or t > 0
            assert v is None or v >= 0
