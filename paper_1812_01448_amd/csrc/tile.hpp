// Device-side contract of the fused K-step kernel: the per-tile record it reads, the
// largest fusion depth, and the XCD-aware mapping of work-groups to tiles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tyee {

constexpr int kMaxFusion = 8;  // largest number of steps one fused launch advances

struct TileInfo {
    int32_t n_core;      // core triangles are local [0, n_core), device slots core_base + l
    int32_t n_own;       // owned edges are local [0, n_own)
    int32_t tri_off;     // offset of this tile in the packed triangle arrays
    int32_t edge_off;    // offset of this tile in the packed edge arrays
    int32_t core_base;   // device slot of the first core triangle
    int32_t own_base;    // device slot of the first owned edge when they are contiguous, else -1
    int32_t cntT[9];     // local triangles with ring level <= m
    int32_t cntE[9];     // local edges with level <= m
};

// Work-groups are dispatched round-robin over the 8 XCDs of the chip (group g runs on
// XCD g mod 8).  Remap so that each XCD works on one contiguous run of groups: the
// neighbour gathers of adjacent groups then hit the same XCD-private L2.
__device__ __forceinline__ int xcd_group(int g, int ngroups) {
    constexpr int kXcd = 8;
    const int q = ngroups / kXcd, r = ngroups % kXcd;
    const int x = g % kXcd, k = g / kXcd;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace tyee
