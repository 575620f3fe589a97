// dls_kernels.hpp -- launch interface between the C ABI and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dlsk {

constexpr int kMaxLevels = 256;

// Per-launch search plan: one descriptor per level of the fill order and the
// set of cells every prefix of the batch assigns.
struct Plan {
    // level descriptor: rsh | rw<<6 | csh<<8 | cw<<14 | onMD<<16 | onAD<<17,
    // rsh/csh = bit offset of the cell's row/column line inside 64-bit word rw/cw
    uint32_t desc[kMaxLevels];
    uint32_t patbits[8];  // bit c set: cell c is assigned in every prefix
    int nlev;             // number of levels (cells the kernels fill)
};

// Work-queue control block of the persistent kernel (device memory).  Each
// field sits on its own 128-byte line: idle waves poll some of them while
// busy waves update others.
struct Ctrl {
    uint64_t head;          // next static task
    uint64_t pad0[15];
    uint64_t dq_reserve;    // donated slots reserved by producers
    uint64_t pad1[15];
    uint64_t dq_head;       // donated slots taken by consumers
    uint64_t pad2[15];
    uint64_t busy;          // waves that may still hold or create work
    uint64_t pad3[15];
    uint64_t hungry;        // idle poller waves waiting for donated work
    uint64_t pad4[15];
    uint64_t sink;          // count target of lanes that have not had a task yet
    uint64_t pad5[15];
};

// Workgroups of each breadth-first expansion kernel.
constexpr int kExBlocks = 1024;

// Device-side state of the breadth-first expansion that deepens a batch too
// small to occupy the GPU before the persistent kernel runs (device memory,
// two of them: pass p reads state p & 1 and writes state (p + 1) & 1).
struct Expand {
    const void *recs;       // current task records
    int64_t num;            // their number
    uint64_t *counts;       // per-task counts written by the search kernel
    const uint32_t *orig;   // task -> prefix index (nullptr: identity)
    uint64_t want;          // sum of candidate counts of the current set
    uint64_t want_next;     // the same for the set being written
    uint64_t nout;          // records written by the pass in progress
    int32_t cur;            // buffer holding the current set: 0 prep, 1 or 2
    int32_t stop;           // nonzero: expansion finished
    uint32_t done;          // workgroups of the pass in progress that finished
    uint32_t pad;
};

struct Tuning {
    int refill_every;  // DFS steps between queue visits
    int steal_depth;   // donate only levels < nlev - steal_depth
    int refill_min;    // idle lanes that trigger a refill while static work remains
    int donate_max;    // donations per wave per queue visit
    int donate_low;    // donate while fewer donated tasks than this are queued
    int tail_poll;     // tail: read the queue state every tail_poll passes (power of 2)
    int chunk_min;     // smallest static chunk a wave takes from the queue
    int lds_masks;     // nonzero: row and column masks in LDS (LdsLane) instead of VGPRs
    int wg_pool;       // tail, VGPR layout: records the waves of a workgroup pool in LDS (0 = off)
};

// Size in bytes of one task record (packed masks of a partial square plus
// level, candidates and origin) for order n; see Rec<> in dls_kernels.hip.
size_t record_bytes(int n, bool vs);

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
    void *records;         // num task records, written by the prep kernel
    int block;
    int grid;
    Ctrl *ctrl;
    void *items;           // donated task records
    uint32_t *ready;       // per donated slot: 1 once published
    int64_t item_cap;
    Tuning tune;
    hipStream_t stream;
    hipEvent_t ev_start;   // recorded around the search kernels when non-null
    hipEvent_t ev_stop;
    // breadth-first expansion of small batches (persistent kernel only;
    // off when ex == nullptr)
    Expand *ex;            // two states
    uint32_t *eblk;        // kExBlocks per-workgroup tallies
    void *ebuf[2];         // ecap task records each
    uint32_t *eorig[2];    // ecap prefix indices each
    uint64_t *tcounts;     // ecap per-task counts
    int64_t ecap;
    int64_t etarget;       // expand while fewer tasks than this
    int epasses;           // expansion passes (each one level deeper)
};

// ---------------------------------------------------------------------------
// serving: one long-running kernel for every order and flags, fed through a
// ring of jobs in host-pinned memory
// ---------------------------------------------------------------------------

// A published job (host-pinned, one per ring slot).  The host writes every
// field, then pub with release; the kernel reads every field with
// system-scope atomic loads, pub first.
struct JobDesc {
    Plan plan;         // the job's fill order
    int32_t n;         // order
    int32_t vs;        // vertical symmetry
    int64_t pre_off;   // byte offset of the job's first workunit in the prefix pool
    uint64_t pub;      // job number << 32 | workunits (each pre_stride(n) bytes); 0 = slot never used
};

// Work state of a job (device memory, one per ring slot, 128 bytes).
struct JobState {
    uint64_t head;       // job number << 32 | workunits taken
    uint64_t remaining;  // pieces not finished: workunits, plus subtrees handed on
    uint64_t total;      // squares counted so far
    uint64_t t_start;    // s_memrealtime when the job was first claimed
    uint64_t claim;      // pub word of the job this state was set up for
    uint64_t dq_res;     // job number << 32 | donation-queue records reserved
    uint64_t dq_head;    // job number << 32 | donation-queue records taken
    uint64_t pad[9];
};

// Result of a job (host-pinned, one per ring slot); pub is written last.
struct JobDone {
    uint64_t pub;
    uint64_t total;
    uint64_t t_start;  // s_memrealtime ticks (100 MHz)
    uint64_t t_end;
    uint64_t shared;   // subtrees handed between waves through the job's donation queue
    uint64_t pad[3];
};

struct ServeArgs {
    int block;
    int grid;
    const JobDesc *jobs;    // host-pinned
    JobState *state;
    JobDone *done;          // host-pinned
    int max_jobs;
    const uint8_t *pool;    // host-pinned prefixes
    const uint32_t *stop;   // host-pinned: nonzero = leave when idle
    const uint64_t *published;  // host-pinned: seq of the last job published
    uint64_t *gate;         // device, zero at launch: [0] waves inside a job | kServeClosing,
                            // [1] tick of the last ring poll, [2] publish word at the last scan,
                            // [3] waves that found no work (they ask busy waves for subtrees)
    uint8_t *items;         // device: a ring of kServeItems donation records of kServeItemBytes per slot
    uint64_t *ready;        // device: kServeItems words per slot (job number << 32 | record state)
    uint32_t *alive;        // host-pinned: one word per wave of the grid, 1 while it runs
    uint64_t idle_ticks;    // the grid leaves once a wave has found no job for this long and none is busy
    int refill_every;
    int chunk;              // most workunits a wave takes from a job at once
    int steal_depth;        // > 0: donate subtrees from levels < levels - steal_depth; else no donation
    hipStream_t stream;
};

constexpr int kServeMinN = 4;
constexpr int kServeMaxN = 9;
constexpr int kServeMaxJobs = 256;
constexpr uint64_t kServeClosing = 1ull << 63;  // gate bit: the grid is leaving
constexpr int kServeItems = 2048;      // entries of a job's donation ring
constexpr int kServeItemBytes = 64;    // >= the largest task record (order 9)
// bytes of one workunit in the prefix pool (n*n cells, padded for 16-byte loads)
inline int pre_stride(int n) { return (n * n + 15) & ~15; }
hipError_t launch_serve(const ServeArgs &a);

uint32_t make_desc(int n, bool vs, int i, int j);
hipError_t launch(const LaunchArgs &a);
hipError_t launch_valu_probe(int blocks, int iters, uint32_t *sink, hipStream_t stream);
hipError_t launch_zero(uint64_t *p, int64_t n, hipStream_t stream);
hipError_t launch_reduce_weighted(const uint64_t *counts, const uint32_t *mult, int64_t num, uint64_t *out,
                                  hipStream_t stream);
size_t lds_bytes(int n, bool vs, int nlev, int block, bool persistent, bool lds_masks = false);

}  // namespace dlsk
