// stage_guard.hpp -- launch geometry of the persistent kernels that stage
// per-block data in the plan's (or batch's) staging region.
//
// A staged kernel addresses its block's slot as stage + blockIdx.x * stride,
// so the region must hold one slot per block of the grid.  The grid of such
// a launch is the occupancy bound, cut to the staging slots the region was
// sized for and to the work items; the host checks, before every staged
// launch, that the region holds that many slots of the launching class's
// stride.  Plain C++ (no HIP) so that it can be checked on the CPU.
#pragma once
#include <cstddef>
#include <cstdint>

namespace mjk {

// Status codes of the class launchers (0 = launched).
enum { kLaunchHip = -1, kLaunchStaging = -2 };

// Blocks of a persistent launch: occupancy x CUs, at most one per staging
// slot when the kernel stages, at most one per work item.  0 means the
// launch cannot run (no slot for a staged kernel, or nothing to do).
inline int64_t persistent_blocks(int64_t occupancy_blocks, int64_t nslot, int64_t nitems, bool staged)
{
    int64_t g = occupancy_blocks;
    if (staged && g > nslot) g = nslot;
    if (g > nitems) g = nitems;
    return g > 0 ? g : 0;
}

// True when `blocks` slots of `slot_doubles` doubles each lie inside a
// staging region of `region_bytes` bytes.
inline bool staging_fits(int64_t blocks, int64_t slot_doubles, size_t region_bytes)
{
    if (blocks < 0 || slot_doubles < 0) return false;
    if (blocks == 0 || slot_doubles == 0) return true;
    const unsigned __int128 need = (unsigned __int128)blocks * (unsigned __int128)slot_doubles * sizeof(double);
    return need <= (unsigned __int128)region_bytes;
}

}  // namespace mjk
