// dls_kernels.hpp -- launch interface between the C ABI and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dlsk {

constexpr int kMaxLevels = 256;

// Per-launch search plan: one descriptor per level of the fill order and the
// set of cells every prefix of the batch assigns.
struct Plan {
    uint32_t desc[kMaxLevels];  // rsh | rw<<5 | csh<<8 | cw<<13 | md<<16 | ad<<17
    uint32_t patbits[8];        // bit c set: cell c is assigned in every prefix
    int nlev;                   // number of levels (cells the kernel fills)
};

// Work-queue control block of the persistent kernel (device memory).
struct Ctrl {
    uint64_t head;         // next static prefix
    uint64_t dq_reserve;   // donated slots reserved by producers
    uint64_t dq_head;      // donated slots taken by consumers
    uint64_t outstanding;  // tasks taken or queued but not finished
    uint64_t pad[4];
};

// A donated subtree: the origin prefix, the values taken at levels
// 0..level-1 (4 bits each) and the candidate set left at `level`.
struct Item {
    uint32_t origin;
    uint16_t level;
    uint16_t cand;
    uint32_t ready;        // 1 once published; consumers reset it to 0
    uint8_t path[52];
};
static_assert(sizeof(Item) == 64, "Item layout");
constexpr int kItemMaxLevels = 104;

struct Tuning {
    int refill_every;  // DFS steps between queue visits
    int steal_depth;   // donate only levels < nlev - steal_depth
    int low_water;     // donate while fewer donated items than this are queued
    int pad;
};

struct LaunchArgs {
    int n;
    bool vs;
    bool persistent;
    Plan plan;
    const uint8_t *prefixes;
    int64_t num;
    uint64_t *counts;
    uint32_t *status;
    uint64_t *steps;
    int block;
    int grid;
    Ctrl *ctrl;
    Item *items;
    int64_t item_cap;
    Tuning tune;
    hipStream_t stream;
};

uint32_t make_desc(int n, int i, int j);
hipError_t launch(const LaunchArgs &a);
hipError_t clear_item_flags(Item *items, int64_t n, hipStream_t stream);
hipError_t launch_valu_probe(int blocks, int iters, uint32_t *sink, hipStream_t stream);
size_t lds_bytes(int n, int nlev, int block);

}  // namespace dlsk
