// dls_api.cpp -- the C ABI declared in include/dls.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dls.h"
#include "dls_canon.hpp"
#include "dls_host.hpp"
#include "dls_kernels.hpp"

namespace {

using dls::kEmpty;

bool valid_n(int n) { return n >= 1 && n <= DLS_MAXN; }

bool valid_cells(int n, const uint8_t *sq) {
    for (int c = 0; c < n * n; ++c)
        if (sq[c] != kEmpty && sq[c] >= n) return false;
    return true;
}

std::vector<uint8_t> identity_prefix(int n) {
    std::vector<uint8_t> p((size_t)n * n, kEmpty);
    for (int j = 0; j < n; ++j) p[j] = (uint8_t)j;
    return p;
}

std::vector<uint8_t> pattern_of(int n, const uint8_t *sq) {
    std::vector<uint8_t> a((size_t)n * n);
    for (int c = 0; c < n * n; ++c) a[c] = sq[c] != kEmpty;
    return a;
}

// hourglass cells that the order lists (left-half representatives with VS)
int hourglass_levels(int n, bool vs, const std::vector<int> &order) {
    std::vector<uint8_t> in((size_t)n * n, 0);
    for (int c : dls::hourglass_cells(n)) in[c] = 1;
    int k = 0;
    for (int c : order) {
        int i = c / n, j = c % n;
        if (in[c] || (vs && in[i * n + (n - 1 - j)])) ++k;
    }
    return k;
}

bool make_spec(int n, uint32_t flags, const uint8_t *base, int depth, dls::SplitSpec &spec,
               std::unique_ptr<dls::HourglassGroup> &group) {
    const bool vs = flags & DLS_VSYM;
    std::vector<uint8_t> assigned = pattern_of(n, base);
    std::vector<int> first;
    if (flags & DLS_SYMBREAK) first = dls::hourglass_cells(n);
    std::vector<int> order = dls::fill_order(n, vs, assigned.data(), first);
    if (depth < 0 || depth > (int)order.size()) return false;
    spec.n = n;
    spec.vs = vs;
    spec.cells.assign(order.begin(), order.begin() + depth);
    spec.group = nullptr;
    spec.hg_level = -1;
    if (flags & DLS_SYMBREAK) {
        int hl = hourglass_levels(n, vs, order);
        if (depth < hl || n < 2) return false;
        group.reset(new dls::HourglassGroup(n));
        spec.group = group.get();
        spec.hg_level = hl;
    }
    return true;
}

// ---------------------------------------------------------------------------
// device resources
// ---------------------------------------------------------------------------

struct QueueSlot {
    dlsk::Ctrl *ctrl = nullptr;
    void *items = nullptr;      // donated task records (kItemCap of the largest size)
    uint32_t *ready = nullptr;  // publication flag per donated slot
    int64_t cap = 0;
    void *records = nullptr;    // task records of the batch in flight on this stream
    size_t records_bytes = 0;
    // search-kernel timing: one event pair per timed launch since the last query
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t ev_used = 0;
    // breadth-first expansion of small batches (allocated on first use)
    dlsk::Expand *ex = nullptr;      // two states
    uint32_t *eblk = nullptr;        // per-workgroup tallies
    void *ebuf[2] = {nullptr, nullptr};
    uint32_t *eorig[2] = {nullptr, nullptr};
    uint64_t *tcounts = nullptr;
    size_t ebuf_bytes = 0;
    int64_t ecap = 0;
    // status word used when the caller passes no d_status (read and cleared by
    // dls_stream_status)
    uint32_t *status = nullptr;
    // set once work on this stream has been captured into a graph: the graph
    // keeps this slot's buffer addresses, so a buffer outgrown later is
    // retired (kept until the process ends) instead of freed
    bool pinned = false;
    std::vector<void *> retired;
};

constexpr size_t kMaxTimed = 1 << 16;

bool capturing(void *stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// hourglass group of one order on one device (table and cell list)
struct CanonTables {
    uint8_t *tab = nullptr;
    uint8_t *hc = nullptr;
    int groups = 0, kcells = 0;
};

// ---------------------------------------------------------------------------
// scratch of the allocation-free entry point (dls_count_async_noalloc)
// ---------------------------------------------------------------------------
// One array per device, allocated with the code object and held until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device array: its device address comes from hipGetSymbolAddress, once per
// device (DeviceState::scratch), and only that address reaches kernels.
constexpr size_t kNoAllocBytes = size_t(128) << 20;
constexpr int64_t kNoAllocItems = 1 << 14;  // donated-record slots
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct DeviceState {
    bool init = false;
    int cus = 0;
    size_t lds_max = 64 * 1024;         // LDS a workgroup may use (160 KiB on gfx950)
    unsigned char *scratch = nullptr;   // device address of `scratch` on this device
    std::map<void *, QueueSlot> slots;  // scratch and work queue per stream
    std::map<int, CanonTables> canon;   // per order
};

std::mutex g_dev_mu;
std::map<int, DeviceState> g_dev;
thread_local std::string g_last_hip;

int hip_fail(hipError_t e, int code) {
    g_last_hip = hipGetErrorName(e);
    g_last_hip += ": ";
    g_last_hip += hipGetErrorString(e);
    return code;
}

constexpr int64_t kItemCap = 1 << 18;
constexpr size_t kMaxRecord = 80;  // largest task record (order 16)

int device_state(DeviceState **out, int *dev_out) {
    int dev = 0;
    hipError_t e0 = hipGetDevice(&dev);
    if (e0 != hipSuccess) return hip_fail(e0, DLS_EDEVICE);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceState &ds = g_dev[dev];
    if (!ds.init) {
        hipDeviceProp_t prop;
        hipError_t e1 = hipGetDeviceProperties(&prop, dev);
        if (e1 != hipSuccess) return hip_fail(e1, DLS_EDEVICE);
        ds.cus = prop.multiProcessorCount;
        if (prop.sharedMemPerBlock > 0) ds.lds_max = prop.sharedMemPerBlock;
        void *sp = nullptr;
        hipError_t e2 = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
        if (e2 != hipSuccess) return hip_fail(e2, DLS_EDEVICE);
        ds.scratch = static_cast<unsigned char *>(sp);
        ds.init = true;
    }
    *out = &ds;
    *dev_out = dev;
    return DLS_OK;
}

// Scratch for one stream: work-queue control block, donated-record slots and
// their flags (allocated once), task records (grown to the largest batch).
int queue_slot(DeviceState *ds, void *stream, size_t records_bytes, QueueSlot **out) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = ds->slots.find(stream);
    const bool cap = capturing(stream);
    if (cap && (it == ds->slots.end() || it->second.records_bytes < records_bytes)) return DLS_ECAPTURE;
    if (it == ds->slots.end()) {
        QueueSlot s;
        if (hipMalloc((void **)&s.ctrl, sizeof(dlsk::Ctrl)) != hipSuccess) return DLS_ENOMEM;
        if (hipMalloc(&s.items, kMaxRecord * kItemCap) != hipSuccess) return DLS_ENOMEM;
        if (hipMalloc((void **)&s.ready, sizeof(uint32_t) * kItemCap) != hipSuccess) return DLS_ENOMEM;
        if (hipMalloc((void **)&s.status, sizeof(uint32_t)) != hipSuccess) return DLS_ENOMEM;
        s.cap = kItemCap;
        hipError_t e2 = hipMemset(s.ctrl, 0, sizeof(dlsk::Ctrl));
        if (e2 == hipSuccess) e2 = hipMemset(s.ready, 0, sizeof(uint32_t) * kItemCap);
        if (e2 == hipSuccess) e2 = hipMemset(s.status, 0, sizeof(uint32_t));
        if (e2 == hipSuccess) e2 = hipDeviceSynchronize();
        if (e2 != hipSuccess) return hip_fail(e2, DLS_EDEVICE);
        it = ds->slots.emplace(stream, s).first;
    }
    QueueSlot &q = it->second;
    if (cap) q.pinned = true;
    if (q.records_bytes < records_bytes) {
        if (q.records && q.pinned) {
            // a captured graph may still use it
            q.retired.push_back(q.records);
            q.records = nullptr;
            q.records_bytes = 0;
        } else if (q.records) {
            // the previous batch on this stream may still be running
            hipError_t e3 = hipStreamSynchronize((hipStream_t)stream);
            if (e3 != hipSuccess) return hip_fail(e3, DLS_EDEVICE);
            (void)hipFree(q.records);
            q.records = nullptr;
            q.records_bytes = 0;
        }
        size_t want = records_bytes + records_bytes / 4;
        if (hipMalloc(&q.records, want) != hipSuccess) return DLS_ENOMEM;
        q.records_bytes = want;
    }
    *out = &q;
    return DLS_OK;
}

// Expansion buffers of a stream for `ecap` tasks of `rb` bytes each.
int expand_buffers(void *stream, QueueSlot *q, int64_t ecap, size_t rb) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    const size_t want = (size_t)ecap * rb;
    if (q->ex && q->ecap >= ecap && q->ebuf_bytes >= want) return DLS_OK;
    if (capturing(stream)) return DLS_ECAPTURE;
    if (q->ex) {
        if (!q->pinned) {
            hipError_t e = hipStreamSynchronize((hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, DLS_EDEVICE);
        }
        for (void *p : {(void *)q->ebuf[0], (void *)q->ebuf[1], (void *)q->eorig[0], (void *)q->eorig[1],
                        (void *)q->tcounts})
            if (p) {
                if (q->pinned) q->retired.push_back(p);  // a captured graph may still use it
                else (void)hipFree(p);
            }
        q->ebuf[0] = q->ebuf[1] = nullptr;
        q->eorig[0] = q->eorig[1] = nullptr;
        q->tcounts = nullptr;
        q->ebuf_bytes = 0;
        q->ecap = 0;
    } else {
        if (hipMalloc((void **)&q->ex, 2 * sizeof(dlsk::Expand)) != hipSuccess) {
            q->ex = nullptr;
            return DLS_ENOMEM;
        }
        if (hipMalloc((void **)&q->eblk, sizeof(uint32_t) * dlsk::kExBlocks) != hipSuccess) {
            (void)hipFree(q->ex);
            q->ex = nullptr;
            q->eblk = nullptr;
            return DLS_ENOMEM;
        }
    }
    for (int k = 0; k < 2; ++k) {
        if (hipMalloc(&q->ebuf[k], want) != hipSuccess) return DLS_ENOMEM;
        if (hipMalloc((void **)&q->eorig[k], sizeof(uint32_t) * (size_t)ecap) != hipSuccess) return DLS_ENOMEM;
    }
    if (hipMalloc((void **)&q->tcounts, sizeof(uint64_t) * (size_t)ecap) != hipSuccess) return DLS_ENOMEM;
    q->ebuf_bytes = want;
    q->ecap = ecap;
    return DLS_OK;
}

// cells == nullptr: the levels follow the fill order of Sec. 2.3 (variant);
// otherwise they are exactly cells[0..ncells) in that order, each empty in
// the pattern (with vs: left-half cells, the mirror implied).
int build_plan(int n, bool vs, const uint8_t *pattern, dlsk::Plan &plan, int variant = 0,
               const int *cells = nullptr, int ncells = 0) {
    std::vector<uint8_t> pat((size_t)n * n, 0);
    if (pattern) {
        for (int c = 0; c < n * n; ++c) pat[c] = pattern[c] ? 1 : 0;
    } else {
        for (int j = 0; j < n; ++j) pat[j] = 1;
    }
    if (vs)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (pat[i * n + j] != pat[i * n + (n - 1 - j)]) return DLS_EINVAL;
    if (variant < 0 || variant >= dls::kOrderVariants) return DLS_EINVAL;
    std::vector<int> order;
    if (cells) {
        if (ncells < 0 || ncells > n * n) return DLS_EINVAL;
        std::vector<uint8_t> seen(pat);
        for (int k = 0; k < ncells; ++k) {
            const int c = cells[k];
            if (c < 0 || c >= n * n || seen[c]) return DLS_EINVAL;
            if (vs && 2 * (c % n) > n - 1) return DLS_EINVAL;
            seen[c] = 1;
            if (vs) seen[(c / n) * n + (n - 1 - c % n)] = 1;
            order.push_back(c);
        }
    } else {
        order = dls::fill_order(n, vs, pat.data(), {}, variant);
    }
    if ((int)order.size() > dlsk::kMaxLevels) return DLS_EINVAL;
    std::memset(&plan, 0, sizeof(plan));
    plan.nlev = (int)order.size();
    for (int k = 0; k < plan.nlev; ++k) plan.desc[k] = dlsk::make_desc(n, vs, order[k] / n, order[k] % n);
    for (int c = 0; c < n * n; ++c)
        if (pat[c]) plan.patbits[c >> 5] |= 1u << (c & 31);
    return DLS_OK;
}

// Carves the scratch of one call out of the static array: the work-queue
// control block, the status word, the donated-record flags and slots (fixed
// offsets, so that a call clears what the previous one left there), then the
// task records and the expansion buffers.
struct NoAllocLayout {
    unsigned char *base;
    size_t off = 0;
    void *take(size_t bytes) {
        off = (off + 255) & ~size_t(255);
        void *p = base + off;
        off += bytes;
        return p;
    }
    size_t left() const {
        const size_t at = (off + 255) & ~size_t(255);
        return at < kNoAllocBytes ? kNoAllocBytes - at : 0;
    }
};

int count_async_impl(int n, uint32_t flags, const uint8_t *pattern, const uint8_t *d_prefixes, int64_t num,
                     uint64_t *d_counts, uint32_t *d_status, void *stream, const dls_launch *launch,
                     uint64_t *d_steps, const int *cells = nullptr, int ncells = 0, bool noalloc = false) {
    if (!valid_n(n) || num < 0 || (flags & ~(uint32_t)(DLS_VSYM | DLS_PLAIN))) return DLS_EINVAL;
    if (num > 0 && (!d_prefixes || !d_counts)) return DLS_EINVAL;
    if (num == 0) return DLS_OK;
    const bool vs = flags & DLS_VSYM;
    hipStream_t st = (hipStream_t)stream;
    dlsk::LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    int rc = (vs && n % 2 == 1 && n > 1) ? DLS_OK
                                          : build_plan(n, vs, pattern, a.plan, launch ? launch->order_variant : 0,
                                                       cells, ncells);
    if (rc) return rc;
    DeviceState *ds = nullptr;
    int dev = 0;
    rc = device_state(&ds, &dev);
    if (rc) return rc;
    if (vs && n % 2 == 1 && n > 1) {
        // no vertically symmetric square of odd order > 1 exists
        hipError_t ez = dlsk::launch_zero(d_counts, num, st);
        return ez == hipSuccess ? DLS_OK : hip_fail(ez, DLS_EDEVICE);
    }
    a.n = n;
    a.vs = vs;
    a.persistent = !(flags & DLS_PLAIN);
    a.prefixes = d_prefixes;
    a.num = num;
    a.counts = d_counts;
    a.status = d_status;
    a.steps = d_steps;
    a.stream = st;
    int block = (launch && launch->block) ? launch->block : 256;
    if (block < 64 || block > 1024 || block % 64) return DLS_EINVAL;
    // line masks in LDS: by default from order 9 on, where the packed VGPR
    // layout needs two words per kind (measured 21-27 % faster there); at
    // N <= 8 the faster layout depends on the workload (autotuner)
    const bool lm = a.persistent && ((launch && launch->lds_masks) ? launch->lds_masks > 0 : n >= 9);
    while (block > 64 && dlsk::lds_bytes(n, vs, a.plan.nlev, block, a.persistent, lm) > ds->lds_max) block /= 2;
    if (dlsk::lds_bytes(n, vs, a.plan.nlev, block, a.persistent, lm) > ds->lds_max) return DLS_EINVAL;
    a.tune.lds_masks = lm ? 1 : 0;
    a.block = block;
    const size_t rb = dlsk::record_bytes(n, vs);
    QueueSlot *qs = nullptr;
    NoAllocLayout na{ds->scratch};
    if (noalloc) {
        // nothing is allocated: every buffer is a piece of the static array
        if (!ds->scratch) return DLS_EDEVICE;
        a.ctrl = static_cast<dlsk::Ctrl *>(na.take(sizeof(dlsk::Ctrl)));
        a.ready = static_cast<uint32_t *>(na.take(sizeof(uint32_t) * kNoAllocItems));
        a.items = na.take(kMaxRecord * kNoAllocItems);
        a.item_cap = kNoAllocItems;
        if ((size_t)num > na.left() / rb) return DLS_ERANGE;
        a.records = na.take(rb * (size_t)num);
    } else {
        rc = queue_slot(ds, stream, rb * (size_t)num, &qs);
        if (rc) return rc;
        a.records = qs->records;
        if (!a.status) a.status = qs->status;  // reported by dls_stream_status
    }
    if (launch && launch->time_kernel) {
        if (noalloc) return DLS_EINVAL;  // the timing events would be allocated
        if (capturing(stream)) return DLS_ECAPTURE;
        std::lock_guard<std::mutex> lk(g_dev_mu);
        if (qs->ev_used == qs->ev.size()) {
            if (qs->ev.size() >= kMaxTimed) return DLS_ERANGE;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            hipError_t ec = hipEventCreate(&e0);
            if (ec == hipSuccess) ec = hipEventCreate(&e1);
            if (ec != hipSuccess) return hip_fail(ec, DLS_EDEVICE);
            qs->ev.emplace_back(e0, e1);
        }
        a.ev_start = qs->ev[qs->ev_used].first;
        a.ev_stop = qs->ev[qs->ev_used].second;
        ++qs->ev_used;
    }
    if (a.persistent) {
        if (!noalloc) {
            a.ctrl = qs->ctrl;
            a.items = qs->items;
            a.ready = qs->ready;
            a.item_cap = qs->cap;
        }
        int bpc = (launch && launch->blocks_per_cu) ? launch->blocks_per_cu : 2048 / block;
        if (bpc < 1) bpc = 1;
        a.grid = ds->cus * bpc;
        a.tune.refill_every = (launch && launch->refill_every) ? launch->refill_every : 32;
        // Work given away across the chip pays for fences; it only pays off when
        // the batch is too small to keep every lane busy (e.g. one big prefix).
        // Inside a wave, idle lanes always take work from busy ones.
        const int64_t lanes = (int64_t)a.grid * block;
        // a batch with fewer tasks than lanes is first deepened on the device
        int64_t et = lanes;
        if (launch && launch->expand_target) et = launch->expand_target < 0 ? 0 : launch->expand_target;
        if (et > (1 << 28)) return DLS_EINVAL;
        if (noalloc && et > num) {
            // the expansion gets what is left of the array: 4 x target slots
            // of two record buffers, two index arrays and one count array
            const size_t fixed = 2 * sizeof(dlsk::Expand) + sizeof(uint32_t) * dlsk::kExBlocks + 6 * 256;
            const size_t per = 4 * (2 * rb + 2 * sizeof(uint32_t) + sizeof(uint64_t));
            const size_t fit = na.left() > fixed ? (na.left() - fixed) / per : 0;
            if ((size_t)et > fit) et = (int64_t)fit;
        }
        const bool expand = et > 0 && num < et && a.plan.nlev >= 3;
        // Global donation (work handed between waves through the device
        // queue) is for batches too small to keep the lanes busy that are not
        // deepened first, e.g. a few huge prefixes with the expansion off.
        int sd = (!expand && num < lanes / 4) ? std::max(8, a.plan.nlev / 3) : 0;
        if (launch && launch->steal_depth) sd = launch->steal_depth < 0 ? 0 : launch->steal_depth;
        a.tune.steal_depth = sd;
        a.tune.refill_min = (launch && launch->refill_min) ? launch->refill_min : 8;
        if (a.tune.refill_min < 1 || a.tune.refill_min > 64) return DLS_EINVAL;
        // the workgroup pool: the kernel caps it at what fits
        a.tune.wg_pool = (launch && launch->wg_pool) ? (launch->wg_pool < 0 ? 0 : launch->wg_pool) : (1 << 20);
        a.tune.donate_max = 2;
        a.tune.donate_low = 256;
        a.tune.tail_poll = 4;
        a.tune.chunk_min = (launch && launch->chunk_min) ? launch->chunk_min : 8;
        if (a.tune.chunk_min < 1 || a.tune.chunk_min > 65536) return DLS_EINVAL;
        if (expand) {
            const int64_t ecap = 4 * et;
            if (noalloc) {
                a.ex = static_cast<dlsk::Expand *>(na.take(2 * sizeof(dlsk::Expand)));
                a.eblk = static_cast<uint32_t *>(na.take(sizeof(uint32_t) * dlsk::kExBlocks));
                a.ebuf[0] = na.take(rb * (size_t)ecap);
                a.ebuf[1] = na.take(rb * (size_t)ecap);
                a.eorig[0] = static_cast<uint32_t *>(na.take(sizeof(uint32_t) * (size_t)ecap));
                a.eorig[1] = static_cast<uint32_t *>(na.take(sizeof(uint32_t) * (size_t)ecap));
                a.tcounts = static_cast<uint64_t *>(na.take(sizeof(uint64_t) * (size_t)ecap));
                if (na.off > kNoAllocBytes) return DLS_ERANGE;  // cannot happen: sized above
            } else {
                rc = expand_buffers(stream, qs, ecap, rb);
                if (rc) return rc;
                a.ex = qs->ex;
                a.eblk = qs->eblk;
                a.ebuf[0] = qs->ebuf[0];
                a.ebuf[1] = qs->ebuf[1];
                a.eorig[0] = qs->eorig[0];
                a.eorig[1] = qs->eorig[1];
                a.tcounts = qs->tcounts;
            }
            a.ecap = ecap;
            a.etarget = et;
            a.epasses = std::min(a.plan.nlev - 2, 16);
        }
    }
    hipError_t e = dlsk::launch(a);
    return e == hipSuccess ? DLS_OK : hip_fail(e, DLS_EDEVICE);
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};


// A node of the breadth-first split below: the line masks of the base plus
// the values placed so far, and those values (the cells are the first levels
// of the order, so the square is rebuilt from the base at the end).
struct SplitNode {
    uint16_t rows[DLS_MAXN], cols[DLS_MAXN], md, ad;
    uint8_t val[64];  // value placed at level t
};
constexpr int kSplitMaxDepth = 64;

// places v at (i, j); false if a row, column or diagonal already holds it
bool split_place(int n, uint16_t *rows, uint16_t *cols, uint16_t &md, uint16_t &ad, int i, int j, int v) {
    const uint16_t b = (uint16_t)(1u << v);
    if ((rows[i] & b) || (cols[j] & b)) return false;
    if (i == j && (md & b)) return false;
    if (i + j == n - 1 && (ad & b)) return false;
    rows[i] |= b;
    cols[j] |= b;
    if (i == j) md |= b;
    if (i + j == n - 1) ad |= b;
    return true;
}

// Workunits of a serving request (Sec. 5.2), breadth-first: the consistent
// assignments of the first d cells of `order` (with vs: left-half cells, each
// with its mirror), for the smallest d that gives at least min_tasks of them
// or d = maxd.  One pass per level, so the cost is that of the levels
// visited.  Empty if the base is inconsistent or no assignment is.
std::vector<uint8_t> serve_split(int n, bool vs, const uint8_t *base, const std::vector<int> &order,
                                 int64_t min_tasks, int maxd) {
    const int nn = n * n;
    maxd = std::min(maxd, kSplitMaxDepth);
    SplitNode root;
    std::memset(&root, 0, sizeof(root));
    for (int c = 0; c < nn; ++c)
        if (base[c] != kEmpty && !split_place(n, root.rows, root.cols, root.md, root.ad, c / n, c % n, base[c]))
            return {};
    std::vector<SplitNode> cur(1, root), next;
    int d = 0;
    for (; d < maxd && (int64_t)cur.size() < min_tasks && !cur.empty(); ++d) {
        const int c = order[d], i = c / n, j = c % n, mj = n - 1 - j;
        next.clear();
        next.reserve(cur.size() * 2);
        const uint16_t all = (uint16_t)((1u << n) - 1u);
        for (const SplitNode &x : cur) {
            // values free at (i, j) before trying them one by one
            uint16_t used = x.rows[i] | x.cols[j];
            if (i == j) used |= x.md;
            if (i + j == n - 1) used |= x.ad;
            for (uint16_t fr = (uint16_t)(all & ~used); fr; fr &= (uint16_t)(fr - 1)) {
                const int v = __builtin_ctz(fr);
                SplitNode y = x;
                if (!split_place(n, y.rows, y.cols, y.md, y.ad, i, j, v)) continue;
                if (vs && mj != j && !split_place(n, y.rows, y.cols, y.md, y.ad, i, mj, n - 1 - v)) continue;
                if (vs && mj == j && 2 * v != n - 1) continue;
                y.val[d] = (uint8_t)v;
                next.push_back(y);
            }
        }
        cur.swap(next);
    }
    std::vector<uint8_t> out(cur.size() * (size_t)nn);
    for (size_t t = 0; t < cur.size(); ++t) {
        uint8_t *q = out.data() + t * nn;
        std::memcpy(q, base, (size_t)nn);
        for (int l = 0; l < d; ++l) {
            const int c = order[l], i = c / n, j = c % n;
            q[c] = cur[t].val[l];
            if (vs && n - 1 - j != j) q[i * n + (n - 1 - j)] = (uint8_t)(n - 1 - cur[t].val[l]);
        }
    }
    return out;
}

int count_host(int n, uint32_t flags, const uint8_t *prefixes, int64_t num, uint64_t *counts_out, const int *cells,
               int ncells) {
    if (!valid_n(n) || num < 0 || (flags & ~(uint32_t)(DLS_VSYM | DLS_PLAIN))) return DLS_EINVAL;
    if (num > 0 && (!prefixes || !counts_out)) return DLS_EINVAL;
    const int nn = n * n;
    for (int64_t k = 0; k < num; ++k)
        if (!valid_cells(n, prefixes + k * nn)) return DLS_EINVAL;
    if (num == 0) return DLS_OK;
    const bool vs = flags & DLS_VSYM;
    std::fill(counts_out, counts_out + num, 0);
    if (vs && n % 2 == 1 && n > 1) return DLS_OK;
    try {
        // group prefixes by which cells they assign (mirror-completed with VS)
        std::map<std::vector<uint8_t>, std::vector<int64_t>> groups;
        std::vector<uint8_t> work((size_t)num * nn);
        for (int64_t k = 0; k < num; ++k) {
            uint8_t *dst = work.data() + k * nn;
            if (vs) {
                if (!dls::vs_complete(n, prefixes + k * nn, dst)) continue;  // count stays 0
            } else {
                std::memcpy(dst, prefixes + k * nn, nn);
            }
            groups[pattern_of(n, dst)].push_back(k);
        }
        if (cells) {
            // reject a bad cell list before touching the device
            dlsk::Plan probe;
            for (auto &g : groups) {
                int rc0 = build_plan(n, vs, g.first.data(), probe, 0, cells, ncells);
                if (rc0) return rc0;
            }
        }
        hipStream_t st = nullptr;
        for (auto &g : groups) {
            const std::vector<int64_t> &ids = g.second;
            const int64_t m = (int64_t)ids.size();
            std::vector<uint8_t> packed((size_t)m * nn);
            for (int64_t t = 0; t < m; ++t) std::memcpy(packed.data() + t * nn, work.data() + ids[t] * nn, nn);
            DevBuf dp, dc, dsb;
            if (hipMalloc(&dp.p, packed.size()) != hipSuccess) return DLS_ENOMEM;
            if (hipMalloc(&dc.p, sizeof(uint64_t) * m) != hipSuccess) return DLS_ENOMEM;
            if (hipMalloc(&dsb.p, sizeof(uint32_t)) != hipSuccess) return DLS_ENOMEM;
            if (hipMemcpy(dp.p, packed.data(), packed.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemset(dsb.p, 0, sizeof(uint32_t)) != hipSuccess)
                return DLS_EDEVICE;
            int rc = count_async_impl(n, flags, g.first.data(), (const uint8_t *)dp.p, m, (uint64_t *)dc.p,
                                      (uint32_t *)dsb.p, st, nullptr, nullptr, cells, ncells);
            if (rc) return rc;
            std::vector<uint64_t> c((size_t)m);
            uint32_t status = 0;
            if (hipStreamSynchronize(st) != hipSuccess ||
                hipMemcpy(c.data(), dc.p, sizeof(uint64_t) * m, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(&status, dsb.p, sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
                return DLS_EDEVICE;
            if (status & ~1u) return DLS_EDEVICE;
            if (status & 1u) return DLS_EPATTERN;
            for (int64_t t = 0; t < m; ++t) counts_out[ids[t]] = c[t];
        }
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

}  // namespace

extern "C" {

const char *dls_strerror(int err) {
    switch (err) {
        case DLS_OK: return "ok";
        case DLS_EINVAL: return "invalid argument";
        case DLS_ERANGE: return "output capacity too small";
        case DLS_ENOMEM: return "out of memory";
        case DLS_EDEVICE: return "HIP device error";
        case DLS_EPATTERN: return "prefix does not match the pattern";
        case DLS_EBUSY: return "no room now: the server's job ring or task pool is full (retry after a job completes)";
        case DLS_ECAPTURE: return "stream is being captured: device memory would have to be allocated "
                                  "(make one uncaptured call with at least as many prefixes on this "
                                  "stream first) or kernel timing was requested";
        default: return "unknown error";
    }
}

const char *dls_version(void) { return "dls-mi355x 1.0 (gfx950)"; }

const char *dls_last_hip_error(void) { return g_last_hip.c_str(); }

int dls_order(int n, uint32_t flags, const uint8_t *assigned, uint8_t *order_out, int *len_out) {
    if (!valid_n(n) || !assigned || !order_out || !len_out) return DLS_EINVAL;
    if (flags & ~(uint32_t)(DLS_VSYM | DLS_SYMBREAK)) return DLS_EINVAL;
    try {
        std::vector<int> first;
        if (flags & DLS_SYMBREAK) first = dls::hourglass_cells(n);
        std::vector<int> o = dls::fill_order(n, flags & DLS_VSYM, assigned, first);
        for (size_t k = 0; k < o.size(); ++k) order_out[k] = (uint8_t)o[k];
        *len_out = (int)o.size();
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_split(int n, uint32_t flags, int depth, uint8_t *prefixes_out, uint32_t *mult_out, int64_t cap,
              int64_t *num_out) {
    if (!valid_n(n) || !num_out || (flags & ~(uint32_t)(DLS_VSYM | DLS_SYMBREAK))) return DLS_EINVAL;
    try {
        std::vector<uint8_t> base = identity_prefix(n);
        dls::SplitSpec spec;
        std::unique_ptr<dls::HourglassGroup> group;
        if (!make_spec(n, flags, base.data(), depth, spec, group)) return DLS_EINVAL;
        if (!prefixes_out) {
            *num_out = dls::split_count(spec, base.data());
            return DLS_OK;
        }
        const int64_t total = dls::split_write(spec, base.data(), prefixes_out, mult_out, cap);
        *num_out = total;
        if (total > cap) return DLS_ERANGE;
        if (mult_out && !(flags & DLS_SYMBREAK)) std::fill(mult_out, mult_out + total, 1u);
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_split_from(int n, uint32_t flags, const uint8_t *base, int depth, uint8_t *prefixes_out, int64_t cap,
                   int64_t *num_out) {
    if (!valid_n(n) || !base || !num_out || (flags & ~(uint32_t)DLS_VSYM)) return DLS_EINVAL;
    if (!valid_cells(n, base)) return DLS_EINVAL;
    try {
        std::vector<uint8_t> b(base, base + n * n);
        if (flags & DLS_VSYM) {
            if (!dls::vs_complete(n, base, b.data())) {
                *num_out = 0;
                return DLS_OK;
            }
        }
        dls::SplitSpec spec;
        std::unique_ptr<dls::HourglassGroup> group;
        if (!make_spec(n, flags, b.data(), depth, spec, group)) return DLS_EINVAL;
        if (!prefixes_out) {
            *num_out = dls::split_count(spec, b.data());
            return DLS_OK;
        }
        int64_t total = dls::split_write(spec, b.data(), prefixes_out, nullptr, cap);
        *num_out = total;
        if (total > cap) return DLS_ERANGE;
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_split_cells(int n, uint32_t flags, const uint8_t *base, const int *cells, int ncells,
                    uint8_t *prefixes_out, int64_t cap, int64_t *num_out) {
    if (!valid_n(n) || !base || !num_out || ncells < 0 || (ncells > 0 && !cells)) return DLS_EINVAL;
    if (flags & ~(uint32_t)DLS_VSYM) return DLS_EINVAL;
    if (!valid_cells(n, base)) return DLS_EINVAL;
    const bool vs = flags & DLS_VSYM;
    try {
        std::vector<uint8_t> b(base, base + n * n);
        if (vs && !dls::vs_complete(n, base, b.data())) {
            *num_out = 0;
            return DLS_OK;
        }
        std::vector<uint8_t> seen((size_t)n * n, 0);
        for (int c = 0; c < n * n; ++c) seen[c] = b[c] != dls::kEmpty;
        dls::SplitSpec spec;
        spec.n = n;
        spec.vs = vs;
        for (int k = 0; k < ncells; ++k) {
            const int c = cells[k];
            if (c < 0 || c >= n * n || seen[c]) return DLS_EINVAL;
            if (vs && 2 * (c % n) > n - 1) return DLS_EINVAL;
            seen[c] = 1;
            if (vs) seen[(c / n) * n + (n - 1 - c % n)] = 1;
            spec.cells.push_back(c);
        }
        if (!prefixes_out) {
            *num_out = dls::split_count(spec, b.data());
            return DLS_OK;
        }
        int64_t total = dls::split_write(spec, b.data(), prefixes_out, nullptr, cap);
        *num_out = total;
        if (total > cap) return DLS_ERANGE;
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_split_target(int n, uint32_t flags, const uint8_t *base, int64_t min_tasks, int max_depth,
                     uint8_t *prefixes_out, int64_t cap, int64_t *num_out) {
    if (!valid_n(n) || !base || !num_out || min_tasks < 1 || max_depth < 0) return DLS_EINVAL;
    if ((flags & ~(uint32_t)DLS_VSYM) || !valid_cells(n, base)) return DLS_EINVAL;
    const bool vs = flags & DLS_VSYM;
    try {
        std::vector<uint8_t> b(base, base + n * n);
        std::vector<uint8_t> units;
        if (!(vs && n % 2 == 1 && n > 1) && (!vs || dls::vs_complete(n, base, b.data()))) {
            const std::vector<uint8_t> assigned = pattern_of(n, b.data());
            const std::vector<int> order = dls::fill_order(n, vs, assigned.data(), {});
            const int maxd = std::min(max_depth, std::max(0, (int)order.size() - 2));
            units = serve_split(n, vs, b.data(), order, min_tasks, maxd);
        }
        const int64_t p = (int64_t)(units.size() / ((size_t)n * n));
        *num_out = p;
        if (!prefixes_out) return DLS_OK;
        if (p > cap) return DLS_ERANGE;
        std::memcpy(prefixes_out, units.data(), units.size());
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_order_cost(int n, uint32_t flags, const int *cells, int ncells, const uint8_t *prefixes, int64_t num,
                   uint64_t *steps_out, uint64_t *leaves_out) {
    if (!valid_n(n) || ncells < 0 || (ncells > 0 && !cells) || num < 0 || (num > 0 && !prefixes)) return DLS_EINVAL;
    if (!steps_out || !leaves_out || (flags & ~(uint32_t)DLS_VSYM)) return DLS_EINVAL;
    const bool vs = flags & DLS_VSYM;
    for (int k = 0; k < ncells; ++k) {
        const int c = cells[k];
        if (c < 0 || c >= n * n) return DLS_EINVAL;
        if (vs && 2 * (c % n) > n - 1) return DLS_EINVAL;
        for (int t = 0; t < k; ++t)
            if (cells[t] == c) return DLS_EINVAL;
    }
    for (int64_t k = 0; k < num; ++k)
        if (!valid_cells(n, prefixes + k * n * n)) return DLS_EINVAL;
    try {
        std::vector<int> order(cells, cells + ncells);
        if (dls::order_cost(n, vs, order, prefixes, num, steps_out, leaves_out)) return DLS_EINVAL;
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_split_sample(int n, uint32_t flags, int depth, const int64_t *indices, int64_t k,
                     uint8_t *prefixes_out, int64_t *total_out) {
    if (!valid_n(n) || !total_out || k < 0 || (k > 0 && (!indices || !prefixes_out))) return DLS_EINVAL;
    if (flags & ~(uint32_t)DLS_VSYM) return DLS_EINVAL;
    for (int64_t t = 0; t < k; ++t)
        if (indices[t] < 0 || (t > 0 && indices[t] <= indices[t - 1])) return DLS_EINVAL;
    try {
        std::vector<uint8_t> base = identity_prefix(n);
        dls::SplitSpec spec;
        std::unique_ptr<dls::HourglassGroup> group;
        if (!make_spec(n, flags, base.data(), depth, spec, group)) return DLS_EINVAL;
        int64_t r = dls::split_select(spec, base.data(), indices, k, prefixes_out);
        if (r < 0) {
            *total_out = -r - 1;
            return DLS_ERANGE;
        }
        *total_out = r;
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int64_t dls_group_order(int n) {
    if (n < 2 || n > DLS_MAXN) return DLS_EINVAL;
    int64_t m = n / 2, r = 2;
    for (int64_t k = 0; k < m; ++k) r *= 2;
    for (int64_t k = 2; k < m; ++k) r *= k;
    return r;
}

int dls_canon(int n, const uint8_t *h, uint32_t *mult_out) {
    if (n < 2 || n > DLS_MAXN || !h || !mult_out || !valid_cells(n, h)) return DLS_EINVAL;
    for (int c : dls::hourglass_cells(n))
        if (h[c] == kEmpty) return DLS_EINVAL;
    for (int j = 0; j < n; ++j)
        if (h[j] != j) return DLS_EINVAL;
    try {
        dls::HourglassGroup g(n);
        *mult_out = g.canon(h);
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_count_async(int n, uint32_t flags, const uint8_t *d_prefixes, int64_t num, uint64_t *d_counts,
                    void *stream) {
    if (!valid_n(n) || num < 0 || (flags & ~(uint32_t)(DLS_VSYM | DLS_PLAIN))) return DLS_EINVAL;
    if (num > 0 && (!d_prefixes || !d_counts)) return DLS_EINVAL;
    if (num == 0) return DLS_OK;
    // the pattern of assigned cells is prefix 0's: one small copy on the
    // caller's stream, which waits for the work queued there before it
    if (capturing(stream)) return DLS_ECAPTURE;
    uint8_t first[DLS_MAXN * DLS_MAXN];
    hipError_t e = hipMemcpyAsync(first, d_prefixes, (size_t)n * n, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, DLS_EDEVICE);
    if (!valid_cells(n, first)) return DLS_EINVAL;
    const std::vector<uint8_t> pat = pattern_of(n, first);
    return count_async_impl(n, flags, pat.data(), d_prefixes, num, d_counts, nullptr, stream, nullptr, nullptr);
}

int dls_count_async_noalloc(int n, uint32_t flags, const uint8_t *pattern, const uint8_t *d_prefixes,
                            int64_t num, uint64_t *d_counts, uint32_t *d_status, void *stream,
                            const dls_launch *launch) {
    if (num > 0 && !d_status) return DLS_EINVAL;
    return count_async_impl(n, flags, pattern, d_prefixes, num, d_counts, d_status, stream, launch, nullptr,
                            nullptr, 0, true);
}

int dls_stream_status(void *stream, uint32_t *status_out) {
    if (!status_out) return DLS_EINVAL;
    DeviceState *ds = nullptr;
    int dev = 0;
    int rc = device_state(&ds, &dev);
    if (rc) return rc;
    uint32_t *word = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        auto it = ds->slots.find(stream);
        if (it != ds->slots.end()) word = it->second.status;
    }
    *status_out = 0;
    if (!word) return DLS_OK;  // nothing was ever counted on this stream
    if (capturing(stream)) return DLS_ECAPTURE;
    uint32_t v = 0;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipMemcpy(&v, word, sizeof(v), hipMemcpyDeviceToHost);
    if (e == hipSuccess && v) e = hipMemset(word, 0, sizeof(v));
    if (e != hipSuccess) return hip_fail(e, DLS_EDEVICE);
    *status_out = v;
    return DLS_OK;
}

int dls_count_async_ex(int n, uint32_t flags, const uint8_t *pattern, const uint8_t *d_prefixes, int64_t num,
                       uint64_t *d_counts, uint32_t *d_status, void *stream, const dls_launch *launch) {
    return count_async_impl(n, flags, pattern, d_prefixes, num, d_counts, d_status, stream, launch, nullptr);
}

int dls_count_async_stats(int n, uint32_t flags, const uint8_t *pattern, const uint8_t *d_prefixes, int64_t num,
                          uint64_t *d_counts, uint32_t *d_status, void *stream, const dls_launch *launch,
                          uint64_t *d_steps) {
    return count_async_impl(n, flags, pattern, d_prefixes, num, d_counts, d_status, stream, launch, d_steps);
}


int dls_count(int n, uint32_t flags, const uint8_t *prefixes, int64_t num, uint64_t *counts_out) {
    return count_host(n, flags, prefixes, num, counts_out, nullptr, 0);
}

int dls_count_cells(int n, uint32_t flags, const int *cells, int ncells, const uint8_t *prefixes, int64_t num,
                    uint64_t *counts_out) {
    if (!cells && ncells) return DLS_EINVAL;
    static const int none = 0;
    return count_host(n, flags, prefixes, num, counts_out, cells ? cells : &none, ncells);
}

int dls_count_cells_async(int n, uint32_t flags, const int *cells, int ncells, const uint8_t *pattern,
                          const uint8_t *d_prefixes, int64_t num, uint64_t *d_counts, uint32_t *d_status,
                          void *stream, const dls_launch *launch) {
    if (!cells && ncells) return DLS_EINVAL;
    static const int none = 0;
    return count_async_impl(n, flags, pattern, d_prefixes, num, d_counts, d_status, stream, launch, nullptr,
                            cells ? cells : &none, ncells);
}

int dls_hourglass_classes_async(int n, const uint8_t *d_designs, int64_t num, uint8_t *d_out, uint32_t *d_mult,
                                int64_t cap, uint64_t *d_count, uint32_t *d_status, void *stream) {
    if (n < 4 || n > 9 || num < 0 || cap < 0 || !d_count || (num > 0 && !d_designs)) return DLS_EINVAL;
    if (cap > 0 && (!d_out || !d_mult)) return DLS_EINVAL;
    if (capturing(stream)) return DLS_ECAPTURE;
    DeviceState *ds = nullptr;
    int dev = 0;
    int rc = device_state(&ds, &dev);
    if (rc) return rc;
    CanonTables *ct = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        auto it = ds->canon.find(n);
        if (it == ds->canon.end()) {
            dls::HourglassGroup g(n);
            std::vector<uint8_t> tab = g.src_table();
            std::vector<uint8_t> hc;
            for (int c : g.cells()) hc.push_back((uint8_t)c);
            CanonTables t;
            t.groups = g.size();
            t.kcells = (int)hc.size();
            if (hipMalloc((void **)&t.tab, tab.size()) != hipSuccess) return DLS_ENOMEM;
            if (hipMalloc((void **)&t.hc, hc.size()) != hipSuccess) return DLS_ENOMEM;
            hipError_t e = hipMemcpy(t.tab, tab.data(), tab.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(t.hc, hc.data(), hc.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, DLS_EDEVICE);
            it = ds->canon.emplace(n, t).first;
        }
        ct = &it->second;
    }
    if (dlsc::canon_lds_bytes(n, ct->groups, ct->kcells) > 64 * 1024) return DLS_EINVAL;
    dlsc::CanonArgs a;
    a.n = n;
    a.designs = d_designs;
    a.num = num;
    a.src_tab = ct->tab;
    a.groups = ct->groups;
    a.kcells = ct->kcells;
    a.hc = ct->hc;
    a.out = d_out;
    a.out_mult = d_mult;
    a.cap = cap;
    a.out_count = reinterpret_cast<unsigned long long *>(d_count);
    a.status = d_status;
    a.stream = (hipStream_t)stream;
    hipError_t e = dlsk::launch_zero(d_count, 1, a.stream);
    if (e == hipSuccess) e = dlsc::launch_canon(a);
    return e == hipSuccess ? DLS_OK : hip_fail(e, DLS_EDEVICE);
}

int dls_kernel_time_ms(void *stream, float *ms_out, int64_t *launches_out) {
    if (!ms_out) return DLS_EINVAL;
    DeviceState *ds = nullptr;
    int dev = 0;
    int rc = device_state(&ds, &dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = ds->slots.find(stream);
    if (it == ds->slots.end() || it->second.ev_used == 0) return DLS_EINVAL;
    QueueSlot &q = it->second;
    double sum = 0.0;
    for (size_t k = 0; k < q.ev_used; ++k) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, q.ev[k].first, q.ev[k].second);
        if (e != hipSuccess) return hip_fail(e, DLS_EDEVICE);
        sum += ms;
    }
    *ms_out = (float)(sum / (double)q.ev_used);
    if (launches_out) *launches_out = (int64_t)q.ev_used;
    q.ev_used = 0;
    return DLS_OK;
}

int dls_order_variant(int n, uint32_t flags, const uint8_t *assigned, int variant, uint8_t *order_out,
                      int *len_out) {
    if (!valid_n(n) || !assigned || !order_out || !len_out) return DLS_EINVAL;
    if (flags & ~(uint32_t)(DLS_VSYM | DLS_SYMBREAK)) return DLS_EINVAL;
    if (variant < 0 || variant >= dls::kOrderVariants) return DLS_EINVAL;
    try {
        std::vector<int> first;
        if (flags & DLS_SYMBREAK) first = dls::hourglass_cells(n);
        std::vector<int> o = dls::fill_order(n, flags & DLS_VSYM, assigned, first, variant);
        for (size_t k = 0; k < o.size(); ++k) order_out[k] = (uint8_t)o[k];
        *len_out = (int)o.size();
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
    return DLS_OK;
}

int dls_reduce_weighted(const uint64_t *d_counts, const uint32_t *d_mult, int64_t num, uint64_t *d_out,
                        void *stream) {
    if (num < 0 || !d_out || (num > 0 && !d_counts)) return DLS_EINVAL;
    hipError_t e = dlsk::launch_reduce_weighted(d_counts, d_mult, num, d_out, (hipStream_t)stream);
    return e == hipSuccess ? DLS_OK : hip_fail(e, DLS_EDEVICE);
}

int dls_valu_probe(int blocks, int iters, uint32_t *d_sink, void *stream) {
    if (blocks < 1 || iters < 0 || !d_sink) return DLS_EINVAL;
    return dlsk::launch_valu_probe(blocks, iters, d_sink, (hipStream_t)stream) == hipSuccess ? DLS_OK
                                                                                             : DLS_EDEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving: one long-running kernel for every order and flags, fed through a
// job ring in host-pinned memory
// ---------------------------------------------------------------------------

struct dls_server {
    int dev = 0;
    int max_jobs = 0;
    int64_t pool_bytes = 0;
    int variant = 0;
    int max_depth = 24;  // deepest host split of a request
    dlsk::ServeArgs args{};
    hipStream_t run = nullptr;
    hipEvent_t ran = nullptr;  // recorded after every launch of the serving kernel
    bool launched = false;
    int64_t launches = 0;
    dlsk::JobDesc *jobs = nullptr;  // host-pinned
    dlsk::JobState *state = nullptr;  // followed by the gate words (device)
    uint64_t *gate = nullptr;
    uint8_t *items = nullptr;       // device: donation queues, kServeItems records per slot
    uint64_t *ready = nullptr;      // device: their ready words
    int64_t shared = 0;             // subtrees handed between waves, over the jobs retired
    dlsk::JobDone *done = nullptr;  // host-pinned
    uint32_t *stop = nullptr;       // host-pinned
    uint32_t *alive = nullptr;      // host-pinned: one word per wave of the grid
    int waves = 0;
    uint8_t *pool = nullptr;        // host-pinned workunit cells
    size_t device_bytes = 0, pinned_bytes = 0;
    std::mutex mu;
    uint64_t next_seq = 1;
    std::map<int64_t, int64_t> free_ranges;  // prefix pool: byte offset -> length
    int64_t pool_free = 0;
    std::vector<int> free_slots;
    struct Job {
        int slot = -1;
        int64_t off = 0, len = 0;
        uint64_t seq = 0;
        uint64_t pub = 0;   // job number << 32 | workunits, as published
        bool done = false;
        uint64_t count = 0, t0 = 0, t1 = 0;
    };
    std::map<int64_t, Job> tickets;
};

namespace {

void server_release(dls_server *s) {
    if (s->state) (void)hipFree(s->state);
    if (s->items) (void)hipFree(s->items);
    if (s->ready) (void)hipFree(s->ready);
    if (s->jobs) (void)hipHostFree(s->jobs);
    if (s->done) (void)hipHostFree(s->done);
    if (s->stop) (void)hipHostFree(s->stop);
    if (s->alive) (void)hipHostFree(s->alive);
    if (s->pool) (void)hipHostFree(s->pool);
    if (s->ran) (void)hipEventDestroy(s->ran);
    if (s->run) (void)hipStreamDestroy(s->run);
    delete s;
}

// (re)launch the serving kernel unless it is running; caller holds s->mu
int server_ensure_running(dls_server *s) {
    if (s->launched) {
        const hipError_t q = hipEventQuery(s->ran);
        if (q == hipErrorNotReady) return DLS_OK;
        if (q != hipSuccess) return hip_fail(q, DLS_EDEVICE);
    }
    // a fresh grid: no wave inside a job or asking for work, the gate open
    hipError_t e = hipMemsetAsync(s->gate, 0, 4 * sizeof(uint64_t), s->run);
    if (e == hipSuccess) e = dlsk::launch_serve(s->args);
    if (e == hipSuccess) e = hipEventRecord(s->ran, s->run);
    if (e != hipSuccess) return hip_fail(e, DLS_EDEVICE);
    s->launched = true;
    ++s->launches;
    return DLS_OK;
}

// first-fit byte range of the prefix pool, or -1
int64_t server_take_range(dls_server *s, int64_t len) {
    for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
        if (it->second < len) continue;
        const int64_t off = it->first, rest = it->second - len;
        s->free_ranges.erase(it);
        if (rest) s->free_ranges[off + len] = rest;
        s->pool_free -= len;
        return off;
    }
    return -1;
}

void server_give_range(dls_server *s, int64_t off, int64_t len) {
    if (len <= 0) return;
    auto it = s->free_ranges.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != s->free_ranges.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s->free_ranges.erase(nx);
    }
    if (it != s->free_ranges.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s->free_ranges.erase(it);
        }
    }
    s->pool_free += len;
}

}  // namespace

extern "C" {

int dls_server_create(int max_jobs, int64_t pool_bytes, const dls_launch *launch, dls_server **out) {
    if (!out) return DLS_EINVAL;
    *out = nullptr;
    if (max_jobs < 1 || max_jobs > dlsk::kServeMaxJobs || pool_bytes < 16 || pool_bytes > (int64_t(1) << 36))
        return DLS_EINVAL;
    const int variant = launch ? launch->order_variant : 0;
    const int bpc = (launch && launch->blocks_per_cu) ? launch->blocks_per_cu : 1;
    const int refill = (launch && launch->refill_every) ? launch->refill_every : 64;
    const int chunk = (launch && launch->chunk_min) ? launch->chunk_min : 64;
    const int steal = launch ? launch->steal_depth : 0;
    if (variant < 0 || variant >= dls::kOrderVariants || bpc < 1 || bpc > 2 || refill < 2 || chunk < 1 ||
        chunk > 65536 || (launch && launch->block && launch->block != 256))
        return DLS_EINVAL;
    DeviceState *ds = nullptr;
    int dev = 0;
    int rc = device_state(&ds, &dev);
    if (rc) return rc;
    dls_server *s = new (std::nothrow) dls_server;
    if (!s) return DLS_ENOMEM;
    s->dev = dev;
    s->max_jobs = max_jobs;
    s->pool_bytes = (pool_bytes + 15) & ~int64_t(15);
    s->variant = variant;
    const size_t state_bytes = sizeof(dlsk::JobState) * max_jobs;
    s->waves = ds->cus * bpc * 4;
    bool ok = hipMalloc((void **)&s->state, state_bytes + 256) == hipSuccess;
    if (ok) s->gate = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(s->state) + state_bytes);
    const size_t item_bytes = (size_t)max_jobs * dlsk::kServeItems * dlsk::kServeItemBytes;
    const size_t ready_bytes = (size_t)max_jobs * dlsk::kServeItems * sizeof(uint64_t);
    ok = ok && hipMalloc((void **)&s->items, item_bytes) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->ready, ready_bytes) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&s->alive, sizeof(uint32_t) * s->waves, hipHostMallocCoherent) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&s->jobs, sizeof(dlsk::JobDesc) * max_jobs, hipHostMallocCoherent) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&s->done, sizeof(dlsk::JobDone) * max_jobs, hipHostMallocCoherent) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&s->stop, sizeof(uint32_t) * 64, hipHostMallocCoherent) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&s->pool, (size_t)s->pool_bytes, hipHostMallocCoherent) == hipSuccess;
    if (!ok) {
        server_release(s);
        return DLS_ENOMEM;
    }
    s->device_bytes = state_bytes + 256 + item_bytes + ready_bytes;
    s->pinned_bytes = (sizeof(dlsk::JobDesc) + sizeof(dlsk::JobDone)) * max_jobs + 256 + (size_t)s->pool_bytes +
                      sizeof(uint32_t) * s->waves;
    std::memset(s->alive, 0, sizeof(uint32_t) * s->waves);
    std::memset(s->jobs, 0, sizeof(dlsk::JobDesc) * max_jobs);
    std::memset(s->done, 0, sizeof(dlsk::JobDone) * max_jobs);
    std::memset(s->stop, 0, sizeof(uint32_t) * 64);
    // the server's own non-blocking stream (default priority): nothing else
    // is ever queued on it, and it never waits for the null stream
    hipError_t e = hipStreamCreateWithFlags(&s->run, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ran, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemsetAsync(s->state, 0, state_bytes + 256, s->run);
    if (e == hipSuccess) e = hipMemsetAsync(s->ready, 0, ready_bytes, s->run);
    if (e == hipSuccess) e = hipStreamSynchronize(s->run);
    if (e != hipSuccess) {
        const int r = hip_fail(e, DLS_EDEVICE);
        server_release(s);
        return r;
    }
    s->free_ranges[0] = s->pool_bytes;
    s->pool_free = s->pool_bytes;
    for (int k = max_jobs - 1; k >= 0; --k) s->free_slots.push_back(k);
    dlsk::ServeArgs &a = s->args;
    a.block = 256;
    a.grid = ds->cus * bpc;
    a.jobs = s->jobs;
    a.state = s->state;
    a.done = s->done;
    a.max_jobs = max_jobs;
    a.pool = s->pool;
    a.stop = s->stop;
    a.published = reinterpret_cast<const uint64_t *>(s->stop + 32);  // its own cache line
    a.gate = s->gate;
    a.items = s->items;
    a.ready = s->ready;
    a.steal_depth = steal;
    a.alive = s->alive;
    a.idle_ticks = 100000000ull / 20;  // 50 ms at 100 MHz
    a.refill_every = refill + (refill & 1);
    a.chunk = chunk;
    a.stream = s->run;
    *out = s;
    return DLS_OK;
}

int dls_server_submit(dls_server *s, int n, uint32_t flags, const uint8_t *prefix, int64_t min_tasks,
                      int64_t *ticket_out) {
    if (!s || !prefix || !ticket_out || min_tasks < 1) return DLS_EINVAL;
    if (n < dlsk::kServeMinN || n > dlsk::kServeMaxN || (flags & ~(uint32_t)DLS_VSYM)) return DLS_EINVAL;
    if (!valid_cells(n, prefix)) return DLS_EINVAL;
    const bool vs = flags & DLS_VSYM;
    std::lock_guard<std::mutex> lk(s->mu);
    dls_server::Job job;
    job.seq = s->next_seq;
    try {
        std::vector<uint8_t> b(prefix, prefix + n * n);
        bool trivial = false;  // the count is 0 without any work
        if (vs && n % 2 == 1) trivial = true;  // no vertically symmetric square of odd order > 1
        if (!trivial && vs && !dls::vs_complete(n, prefix, b.data())) trivial = true;
        std::vector<uint8_t> units;
        int64_t p = 0;
        if (!trivial) {
            // the shallowest split with at least min_tasks workunits, at most
            // max_depth cells deep, keeping at least two levels for the search
            const std::vector<uint8_t> assigned = pattern_of(n, b.data());
            const std::vector<int> order = dls::fill_order(n, vs, assigned.data(), {}, s->variant);
            const int maxd = std::min(s->max_depth, std::max(0, (int)order.size() - 2));
            units = serve_split(n, vs, b.data(), order, min_tasks, maxd);
            p = (int64_t)(units.size() / ((size_t)n * n));
            if (p == 0) trivial = true;
        }
        if (trivial) {
            job.done = true;
            s->tickets[(int64_t)job.seq] = job;
            *ticket_out = (int64_t)job.seq;
            ++s->next_seq;
            return DLS_OK;
        }
        const int64_t ps = dlsk::pre_stride(n);
        if (p * ps > s->pool_bytes || p > (int64_t)0xFFFFFFFF) return DLS_ERANGE;
        if (s->free_slots.empty()) return DLS_EBUSY;
        const int64_t off = server_take_range(s, p * ps);
        if (off < 0) return DLS_EBUSY;
        const size_t nn = (size_t)n * n;
        dlsk::Plan plan;
        const int rc = build_plan(n, vs, pattern_of(n, units.data()).data(), plan, s->variant);
        if (rc) {
            server_give_range(s, off, p * ps);
            return rc;
        }
        uint8_t *dst = s->pool + off;
        for (int64_t t = 0; t < p; ++t) {
            std::memcpy(dst + t * ps, units.data() + t * nn, nn);
            std::memset(dst + t * ps + nn, 0xFF, (size_t)(ps - (int64_t)nn));
        }
        job.slot = s->free_slots.back();
        s->free_slots.pop_back();
        job.off = off;
        job.len = p * ps;
        dlsk::JobDesc *jd = &s->jobs[job.slot];
        jd->plan = plan;
        jd->n = n;
        jd->vs = vs ? 1 : 0;
        jd->pre_off = off;
        // publish: everything above before the pub word (job number and
        // size), then the counter idle waves watch
        job.pub = ((uint64_t)(job.seq & 0xFFFFFFFFu) << 32) | (uint64_t)p;
        __atomic_store_n(&jd->pub, job.pub, __ATOMIC_RELEASE);
        __atomic_store_n(reinterpret_cast<uint64_t *>(s->stop + 32), job.pub, __ATOMIC_RELEASE);
        s->tickets[(int64_t)job.seq] = job;
        *ticket_out = (int64_t)job.seq;
        ++s->next_seq;
        return server_ensure_running(s);
    } catch (const std::bad_alloc &) {
        return DLS_ENOMEM;
    }
}

int dls_server_poll(dls_server *s, int64_t ticket, uint64_t *count_out, uint64_t *ticks_out, int *done_out) {
    if (!s || !done_out) return DLS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return DLS_EINVAL;
    dls_server::Job &j = it->second;
    if (!j.done) {
        const dlsk::JobDone *d = &s->done[j.slot];
        if (__atomic_load_n(&d->pub, __ATOMIC_ACQUIRE) == j.pub) {
            j.count = __atomic_load_n(&d->total, __ATOMIC_RELAXED);
            j.t0 = __atomic_load_n(&d->t_start, __ATOMIC_RELAXED);
            j.t1 = __atomic_load_n(&d->t_end, __ATOMIC_RELAXED);
            s->shared += (int64_t)__atomic_load_n(&d->shared, __ATOMIC_RELAXED);
            j.done = true;
            server_give_range(s, j.off, j.len);
            s->free_slots.push_back(j.slot);
        } else {
            // the kernel leaves after a while without work; a job published
            // just as it left is served by the next launch
            const int rc = server_ensure_running(s);
            if (rc) return rc;
        }
    }
    *done_out = j.done ? 1 : 0;
    if (j.done) {
        if (count_out) *count_out = j.count;
        if (ticks_out) {
            ticks_out[0] = j.t0;
            ticks_out[1] = j.t1;
        }
        s->tickets.erase(it);
    }
    return DLS_OK;
}

int dls_server_info(dls_server *s, int64_t *allocated_bytes, int64_t *pool_free, int *slots_free,
                    int64_t *launches) {
    if (!s) return DLS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (allocated_bytes) *allocated_bytes = (int64_t)(s->device_bytes + s->pinned_bytes);
    if (pool_free) *pool_free = s->pool_free;
    if (slots_free) *slots_free = (int)s->free_slots.size();
    if (launches) *launches = s->launches;
    return DLS_OK;
}

int dls_server_waves(dls_server *s, int *live_out, int *grid_out) {
    if (!s) return DLS_EINVAL;
    int live = 0;
    for (int w = 0; w < s->waves; ++w) live += __atomic_load_n(&s->alive[w], __ATOMIC_RELAXED) ? 1 : 0;
    if (live_out) *live_out = live;
    if (grid_out) *grid_out = s->waves;
    return DLS_OK;
}

int dls_server_shared(dls_server *s, int64_t *subtrees_out) {
    if (!s || !subtrees_out) return DLS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *subtrees_out = s->shared;
    return DLS_OK;
}

int dls_server_destroy(dls_server *s) {
    if (!s) return DLS_EINVAL;
    int rc = DLS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        __atomic_store_n(&s->stop[0], 1u, __ATOMIC_RELEASE);
        // the kernel sees the flag within its idle backoff; bounded wait
        if (s->launched) {
            for (int t = 0;; ++t) {
                const hipError_t q = hipEventQuery(s->ran);
                if (q == hipSuccess) break;
                if (q != hipErrorNotReady || t > 20000) {
                    rc = DLS_EDEVICE;
                    break;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(500));
            }
        }
    }
    if (rc == DLS_OK) server_release(s);  // else the kernel may still run: leak rather than free
    return rc;
}

}  // extern "C"
