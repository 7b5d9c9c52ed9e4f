"""The launch geometry of staged persistent kernels (csrc/stage_guard.hpp),
compiled with g++ and checked on the CPU.

A staged kernel's block writes its slot at stage + blockIdx.x * stride, so a
launch with more blocks than the staging region holds slots writes past the
region (the workspace's last region, so into whatever memory follows it).
The gradient kernel (dd|dd) was once launched with 2304 blocks (9 per CU x
256 CUs) on an 8-atom input whose plan sized the staging for far fewer slots;
under the launch rule the library uses, that grid is cut to the slots and the
items, and the host refuses a launch whose blocks would not fit the region.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2412_13203_amd", "csrc")

PROG = r"""
#include <cstdio>
#include "stage_guard.hpp"
using namespace mjk;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); return 1; } } while (0)
int main()
{
    // (dd|dd) gradient: its largest split shifted class (fd|dd) has 46 x 31 = 1426
    // accumulators; the slot of one block is that many doubles per lane x 64 lanes
    const long slot = 1426L * 64;
    const long nslot = 72;                     // what a small plan sizes its staging for
    const size_t region = sizeof(double) * slot * nslot;
    // the faulting launch: 2304 blocks against 72 slots
    CHECK(!staging_fits(2304, slot, region));
    // the launch rule: occupancy bound cut to slots and items
    CHECK(persistent_blocks(2304, nslot, 36, true) == 36);
    CHECK(persistent_blocks(2304, nslot, 5000, true) == nslot);
    CHECK(persistent_blocks(2304, nslot, 5000, false) == 2304);   // unstaged kernels are not cut
    CHECK(persistent_blocks(2304, 0, 5000, true) == 0);            // no slot: no launch
    CHECK(persistent_blocks(2304, nslot, 0, true) == 0);
    CHECK(staging_fits(persistent_blocks(2304, nslot, 5000, true), slot, region));
    CHECK(staging_fits(nslot, slot, region));
    CHECK(!staging_fits(nslot + 1, slot, region));
    CHECK(staging_fits(0, slot, 0));
    CHECK(staging_fits(5, 0, 0));
    CHECK(!staging_fits(-1, slot, region));
    // no overflow in the product
    CHECK(!staging_fits(1L << 40, 1L << 40, (size_t)-1));
    std::printf("ok\n");
    return 0;
}
"""


def test_stage_guard(tmp_path):
    src = tmp_path / "guard.cpp"
    exe = tmp_path / "guard"
    src.write_text(PROG)
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", HDR, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
