// dls_kernels.hip -- gfx950 kernels that count diagonal Latin squares.
//
// Each lane runs its own depth-first search over one workunit (Sec. 5.2):
// the bit-arithmetic loop of Alg. 4 (Sec. 3).  On entering a cell the
// forbidden set is CR = Rows[i] | Columns[j] (| MD | AD on the diagonals) and
// the candidates are L = AllN ^ CR; candidates are taken lowest bit first
// (b = L & -L) and marked in / cleared from the masks.  The last cell of the
// order is not entered: its candidate count is added directly.
//
// GPU form of that loop:
//  * the 2N+2 line masks live in VGPRs, packed floor(32/N) lines per word;
//    the cell of the current level selects the word and shift (a per-level
//    descriptor table in LDS, uniform for the whole launch);
//  * the per-lane stack holds, per level, the candidate set at the time the
//    level was left downwards (the taken value is its lowest bit); it is
//    kept in LDS, one row per level, lanes side by side (conflict-free);
//  * one DFS step is the same instruction stream for every lane: either go
//    down one level (take the lowest candidate) or go up one level (clear the
//    value taken there and resume with the remaining candidates).  Marking and
//    clearing are both XOR, so both directions share one code path and lanes
//    at different depths stay converged.
//
// Vertical symmetry (Sec. 5.4): only the left half is searched; placing v at
// (i,j) also places N-1-v at (i,N-1-j).  Row masks receive both values,
// column masks are kept for the left half only (the right half mirrors them),
// and a value on one diagonal puts its mirror on the other.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dls_kernels.hpp"

namespace dlsk {

// ---------------------------------------------------------------------------
// geometry of the packed masks
// ---------------------------------------------------------------------------

template <int N>
struct Geo {
    static constexpr int LPW = 32 / N;                 // lines per 32-bit word
    static constexpr int W = (N + LPW - 1) / LPW;      // words per set of N lines
    static constexpr uint32_t ALL = (N == 32) ? 0xFFFFFFFFu : ((1u << N) - 1u);
};

// descriptor fields (see make_desc on the host side)
__device__ __forceinline__ uint32_t d_rsh(uint32_t d) { return d & 31u; }
__device__ __forceinline__ uint32_t d_rw(uint32_t d) { return (d >> 5) & 7u; }
__device__ __forceinline__ uint32_t d_csh(uint32_t d) { return (d >> 8) & 31u; }
__device__ __forceinline__ uint32_t d_cw(uint32_t d) { return (d >> 13) & 7u; }
__device__ __forceinline__ uint32_t d_md(uint32_t d) { return 0u - ((d >> 16) & 1u); }
__device__ __forceinline__ uint32_t d_ad(uint32_t d) { return 0u - ((d >> 17) & 1u); }

template <int W>
__device__ __forceinline__ uint32_t pick(const uint32_t (&x)[W], uint32_t w) {
    uint32_t r = x[0];
#pragma unroll
    for (int k = 1; k < W; ++k) r = (w == (uint32_t)k) ? x[k] : r;
    return r;
}

template <int W>
__device__ __forceinline__ void flip(uint32_t (&x)[W], uint32_t w, uint32_t bits) {
#pragma unroll
    for (int k = 0; k < W; ++k) x[k] ^= (w == (uint32_t)k) ? bits : 0u;
}

template <int N, bool VS>
struct Lane {
    static constexpr int W = Geo<N>::W;
    uint32_t R[W];     // row masks
    uint32_t C[W];     // column masks (left half only with VS)
    uint32_t md, ad;   // diagonal masks
    uint32_t cand;     // remaining candidates at the current level
    uint32_t cur;      // descriptor of the current level's cell
    int d;             // current level
    int start;         // level at which this lane's task began
    uint64_t cnt;      // completed squares found by this task

    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int k = 0; k < W; ++k) R[k] = C[k] = 0u;
        md = ad = 0u;
        cnt = 0;
    }

    // forbidden values of the cell described by `desc`, as candidates
    __device__ __forceinline__ uint32_t cands(uint32_t desc) const {
        uint32_t cr = pick<W>(R, d_rw(desc)) >> d_rsh(desc);
        cr |= pick<W>(C, d_cw(desc)) >> d_csh(desc);
        cr |= (md & d_md(desc)) | (ad & d_ad(desc));
        return Geo<N>::ALL & ~cr;
    }

    // mark (or clear: XOR) value bit b at the cell described by `desc`
    __device__ __forceinline__ void toggle(uint32_t desc, uint32_t b) {
        const uint32_t mdm = d_md(desc), adm = d_ad(desc);
        if constexpr (VS) {
            // mirror value N-1-v of the lowest set bit v of b (b is one-hot or 0)
            const uint32_t rb = b ? ((1u << (N - 1)) >> __builtin_ctz(b)) : 0u;
            flip<W>(R, d_rw(desc), (b | rb) << d_rsh(desc));
            flip<W>(C, d_cw(desc), b << d_csh(desc));
            md ^= (b & mdm) | (rb & adm);
            ad ^= (b & adm) | (rb & mdm);
        } else {
            flip<W>(R, d_rw(desc), b << d_rsh(desc));
            flip<W>(C, d_cw(desc), b << d_csh(desc));
            md ^= b & mdm;
            ad ^= b & adm;
        }
    }

    __device__ __forceinline__ bool done() const { return cand == 0u && d == start; }

    // One DFS step.  Requires !done().  `desc`: per-level descriptors (LDS);
    // `stk`: this lane's stack slot for level 0, levels `stride` apart.
    template <class S>
    __device__ __forceinline__ void step(const uint32_t *desc, S *stk, int stride, int last) {
        const bool up = (cand == 0u);
        const int nd = up ? d - 1 : d + 1;
        const uint32_t ndesc = desc[nd];
        const uint32_t saved = stk[(up ? d - 1 : d) * stride];
        const uint32_t stored = up ? saved : cand;
        const uint32_t b = stored & (0u - stored);
        toggle(up ? ndesc : cur, b);
        if (!up) stk[d * stride] = (S)cand;
        uint32_t nc = cands(ndesc);
        if (nd == last) {               // last cell: count its candidates
            cnt += (uint64_t)__builtin_popcount(nc);
            nc = 0u;
        }
        cand = up ? (stored ^ b) : nc;
        cur = ndesc;
        d = nd;
    }

    // Load a prefix (n*n bytes in registers-sized chunks from global memory)
    // and check it against the pattern.  Returns false if it breaks a
    // constraint (count 0); sets *mismatch if it does not fit the pattern.
    __device__ __forceinline__ bool load(const uint8_t *sq, const uint32_t *patbits,
                                         bool *mismatch) {
        clear();
        uint32_t bad = 0u, mis = 0u;
        // the whole square is read as dwords; cells are unpacked at
        // compile-time offsets
        constexpr int NN = N * N;
        constexpr int NW = (NN + 3) / 4;
        uint32_t words[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            uint32_t w = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = 4 * k + t;
                if (c < NN) w |= (uint32_t)sq[c] << (8 * t);
            }
            words[k] = w;
        }
#pragma unroll
        for (int c = 0; c < NN; ++c) {
            const int i = c / N, j = c % N;
            const uint32_t v = (words[c >> 2] >> (8 * (c & 3))) & 0xFFu;
            const bool inpat = (patbits[c >> 5] >> (c & 31)) & 1u;
            const bool filled = v != 0xFFu;
            mis |= (inpat != filled) || (filled && v >= (uint32_t)N);
            if (!inpat || !filled || v >= (uint32_t)N) continue;
            if constexpr (VS) {
                if (2 * j > N - 1) continue;   // right half: checked via its mirror
                const int mc = i * N + (N - 1 - j);
                const uint32_t w = (words[mc >> 2] >> (8 * (mc & 3))) & 0xFFu;
                bad |= (w != (uint32_t)(N - 1) - v) ? 1u : 0u;
                const uint32_t b = 1u << v, rb = 1u << (N - 1 - v);
                const int rw = i / Geo<N>::LPW, rs = (i % Geo<N>::LPW) * N;
                const int cw = j / Geo<N>::LPW, cs = (j % Geo<N>::LPW) * N;
                const uint32_t rbits = (b | rb) << rs, cbits = b << cs;
                bad |= (R[rw] & rbits) | (C[cw] & cbits);
                if (2 * j == N - 1) bad |= 1u;  // odd order: middle column impossible
                R[rw] |= rbits;
                C[cw] |= cbits;
                if (i == j) {
                    bad |= (md & b) | (ad & rb);
                    md |= b;
                    ad |= rb;
                }
                if (i + j == N - 1) {
                    bad |= (ad & b) | (md & rb);
                    ad |= b;
                    md |= rb;
                }
            } else {
                const uint32_t b = 1u << v;
                const int rw = i / Geo<N>::LPW, rs = (i % Geo<N>::LPW) * N;
                const int cw = j / Geo<N>::LPW, cs = (j % Geo<N>::LPW) * N;
                const uint32_t rbits = b << rs, cbits = b << cs;
                bad |= (R[rw] & rbits) | (C[cw] & cbits);
                R[rw] |= rbits;
                C[cw] |= cbits;
                if (i == j) {
                    bad |= md & b;
                    md |= b;
                }
                if (i + j == N - 1) {
                    bad |= ad & b;
                    ad |= b;
                }
            }
        }
        *mismatch = mis != 0u;
        return bad == 0u && mis == 0u;
    }

    // Start a task at level `lvl` (all levels below it already applied).
    __device__ __forceinline__ void begin(const uint32_t *desc, int lvl, int nlev, uint32_t c) {
        start = d = lvl;
        cur = desc[lvl];
        cand = c;
        if (lvl == nlev - 1) {
            cnt += (uint64_t)__builtin_popcount(cand);
            cand = 0u;
        }
    }
};

// stack element type: 8 bits suffice up to N = 8
template <int N>
using StackT = typename std::conditional<(N <= 8), uint8_t, uint16_t>::type;

// ---------------------------------------------------------------------------
// plain kernel: one prefix per lane, run to completion
// ---------------------------------------------------------------------------

template <int N, bool VS, bool STATS>
__global__ void __launch_bounds__(1024) plain_kernel(const Plan plan, const uint8_t *__restrict__ prefixes,
                                                     int64_t num, uint64_t *__restrict__ counts,
                                                     uint32_t *status, uint64_t *steps) {
    using S = StackT<N>;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *sdesc = reinterpret_cast<uint32_t *>(smem);
    S *sstk = reinterpret_cast<S *>(smem + sizeof(uint32_t) * kMaxLevels);
    const int nlev = plan.nlev;
    for (int k = threadIdx.x; k < nlev; k += blockDim.x) sdesc[k] = plan.desc[k];
    __syncthreads();

    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= num) return;
    Lane<N, VS> L;
    bool mismatch = false;
    const bool ok = L.load(prefixes + idx * (N * N), plan.patbits, &mismatch);
    if (mismatch && status) atomicOr(status, 1u);
    uint64_t nsteps = 0;
    if (nlev == 0) {
        L.cnt = ok ? 1u : 0u;
    } else if (ok) {
        L.begin(sdesc, 0, nlev, L.cands(sdesc[0]));
        S *stk = sstk + threadIdx.x;
        const int stride = blockDim.x;
        while (!L.done()) {
            L.step(sdesc, stk, stride, nlev - 1);
            if (STATS) ++nsteps;
        }
    }
    counts[idx] = L.cnt;
    if (STATS && steps) atomicAdd((unsigned long long *)steps, (unsigned long long)nsteps);
}

// ---------------------------------------------------------------------------
// persistent kernel: global queue of prefixes + donated subtrees
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// broadcast a 64-bit value from a (wave-uniform) lane
__device__ __forceinline__ uint64_t bcast64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// s_memrealtime ticks at 100 MHz
constexpr uint64_t kStallTicks = 100000000ull * 20;  // 20 s without any queue progress

template <int N, bool VS, bool STATS>
__global__ void __launch_bounds__(1024) persistent_kernel(const Plan plan, const uint8_t *__restrict__ prefixes,
                                                          int64_t num, uint64_t *__restrict__ counts,
                                                          uint32_t *status, uint64_t *steps,
                                                          Ctrl *ctrl, Item *items, int64_t item_cap,
                                                          Tuning tune) {
    using S = StackT<N>;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *sdesc = reinterpret_cast<uint32_t *>(smem);
    S *sstk = reinterpret_cast<S *>(smem + sizeof(uint32_t) * kMaxLevels);
    const int nlev = plan.nlev;
    for (int k = threadIdx.x; k < nlev; k += blockDim.x) sdesc[k] = plan.desc[k];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    S *stk = sstk + threadIdx.x;
    const int stride = blockDim.x;
    const int last = nlev - 1;
    const uint64_t cap = (uint64_t)item_cap;

    Lane<N, VS> L;
    L.cand = 0u;
    L.d = L.start = 0;
    L.cnt = 0;
    bool has = false;          // lane holds a task (possibly finished)
    uint32_t origin = 0;
    bool static_left = true;   // wave-uniform: static prefixes may remain
    uint64_t nsteps = 0;
    uint64_t seen_sig = ~0ull, seen_at = 0;

    for (;;) {
        // ---------------- retire finished tasks ----------------
        if (has && L.done()) {
            if (L.cnt) atomicAdd((unsigned long long *)&counts[origin], (unsigned long long)L.cnt);
            atomicAdd((unsigned long long *)&ctrl->outstanding, ~0ull);  // -1
            has = false;
            L.cnt = 0;
        }
        // ---------------- refill from the static queue (one atomic per wave) ----------------
        uint64_t want = __ballot(!has);
        if (want && static_left) {
            const uint32_t k = (uint32_t)__popcll(want);
            const int leader = __ffsll((unsigned long long)want) - 1;
            uint64_t base = 0;
            if (lane == leader) base = atomicAdd((unsigned long long *)&ctrl->head, (unsigned long long)k);
            base = bcast64(base, leader);
            if (base + k >= (uint64_t)num) static_left = false;
            if (!has) {
                const uint64_t rank = (uint64_t)__popcll(want & ((1ull << lane) - 1ull));
                const uint64_t id = base + rank;
                if (id < (uint64_t)num) {
                    bool mismatch = false;
                    origin = (uint32_t)id;
                    has = true;
                    const bool ok = L.load(prefixes + id * (N * N), plan.patbits, &mismatch);
                    if (mismatch && status) atomicOr(status, 1u);
                    L.cand = 0u;
                    L.d = L.start = 0;
                    if (nlev == 0)
                        L.cnt = ok ? 1u : 0u;
                    else if (ok)
                        L.begin(sdesc, 0, nlev, L.cands(sdesc[0]));
                }
            }
            want = __ballot(!has);
        }
        // ---------------- refill from donated subtrees ----------------
        if (want && !static_left) {
            const uint32_t k = (uint32_t)__popcll(want);
            const int leader = __ffsll((unsigned long long)want) - 1;
            uint64_t h0 = 0, got = 0;
            if (lane == leader) {
                uint64_t h = ld_relaxed(&ctrl->dq_head);
                for (int tries = 0; tries < 64; ++tries) {
                    uint64_t r = ld_relaxed(&ctrl->dq_reserve);
                    if (r > cap) r = cap;
                    const uint64_t avail = r > h ? r - h : 0;
                    if (avail == 0) break;
                    const uint64_t take = avail < k ? avail : k;
                    if (__hip_atomic_compare_exchange_strong(&ctrl->dq_head, &h, h + take, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        h0 = h;
                        got = take;
                        break;
                    }
                }
            }
            h0 = bcast64(h0, leader);
            got = bcast64(got, leader);
            if (!has) {
                const uint64_t rank = (uint64_t)__popcll(want & ((1ull << lane) - 1ull));
                if (rank < got) {
                    Item *it = items + (h0 + rank);
                    // the slot was reserved by a running lane that publishes it
                    // right after writing it; the wait is bounded all the same
                    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                    bool ready = false;
                    for (;;) {
                        if (__hip_atomic_load(&it->ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                            ready = true;
                            break;
                        }
                        if (__builtin_amdgcn_s_memrealtime() - t0 > kStallTicks) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    if (!ready) {
                        if (status) atomicOr(status, 2u);
                        atomicAdd((unsigned long long *)&ctrl->outstanding, ~0ull);
                    } else {
                        __threadfence();
                        origin = it->origin;
                        const int lvl = it->level;
                        const uint32_t icand = it->cand;
                        bool mismatch = false;
                        L.load(prefixes + (uint64_t)origin * (N * N), plan.patbits, &mismatch);
                        for (int l = 0; l < lvl; ++l) {
                            const uint32_t v = ((uint32_t)it->path[l >> 1] >> (4 * (l & 1))) & 15u;
                            const uint32_t b = 1u << v;
                            L.toggle(sdesc[l], b);
                            stk[l * stride] = (S)b;
                        }
                        __hip_atomic_store(&it->ready, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        L.cnt = 0;
                        L.begin(sdesc, lvl, nlev, icand);
                        has = true;
                    }
                }
            }
            want = __ballot(!has);
        }
        // ---------------- termination ----------------
        if (want == __ballot(true) && !static_left) {
            // every lane of this wave is idle and nothing could be taken
            const uint64_t out = ld_relaxed(&ctrl->outstanding);
            if (out == 0) break;
            const uint64_t sig = out ^ (ld_relaxed(&ctrl->dq_reserve) << 20) ^ (ld_relaxed(&ctrl->dq_head) << 40);
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (sig != seen_sig) {
                seen_sig = sig;
                seen_at = now;
            } else if (now - seen_at > kStallTicks) {
                if (lane == 0 && status) atomicOr(status, 2u);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        // ---------------- donate untried siblings when the queue runs dry ----------------
        if (!static_left && has && !L.done() && cap > 0) {
            const uint64_t r = ld_relaxed(&ctrl->dq_reserve);
            const uint64_t h = ld_relaxed(&ctrl->dq_head);
            if (r < cap && r - h < (uint64_t)tune.low_water) {
                // shallowest stacked level with untried candidates
                int lvl = -1;
                const int lim = nlev - tune.steal_depth;
                for (int l = L.start; l < L.d && l < lim; ++l) {
                    const uint32_t s = stk[l * stride];
                    if (s & (s - 1u)) {
                        lvl = l;
                        break;
                    }
                }
                if (lvl >= 0) {
                    const uint64_t slot = atomicAdd((unsigned long long *)&ctrl->dq_reserve, 1ull);
                    if (slot < cap) {
                        atomicAdd((unsigned long long *)&ctrl->outstanding, 1ull);
                        const uint32_t s = stk[lvl * stride];
                        const uint32_t b = s & (0u - s);
                        Item *it = items + slot;
                        it->origin = origin;
                        it->level = (uint16_t)lvl;
                        it->cand = (uint16_t)(s ^ b);
                        for (int l = 0; l < lvl; l += 2) {
                            uint32_t v = (uint32_t)__builtin_ctz((uint32_t)stk[l * stride]);
                            if (l + 1 < lvl) v |= (uint32_t)__builtin_ctz((uint32_t)stk[(l + 1) * stride]) << 4;
                            it->path[l >> 1] = (uint8_t)v;
                        }
                        stk[lvl * stride] = (S)b;
                        __threadfence();
                        __hip_atomic_store(&it->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }
        // ---------------- search ----------------
        for (int it = 0; it < tune.refill_every; ++it) {
            if (has && !L.done()) {
                L.step(sdesc, stk, stride, last);
                if (STATS) ++nsteps;
            }
        }
    }
    if (STATS && steps) atomicAdd((unsigned long long *)steps, (unsigned long long)nsteps);
}

__global__ void reset_ctrl(Ctrl *ctrl, uint64_t num, uint64_t *counts, int64_t ncounts, uint32_t *status) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        ctrl->head = 0;
        ctrl->dq_reserve = 0;
        ctrl->dq_head = 0;
        ctrl->outstanding = num;
    }
    for (int64_t k = t; k < ncounts; k += (int64_t)gridDim.x * blockDim.x) counts[k] = 0;
}

// ready flags of the slots the previous launch on this queue reserved (all
// consumed after a normal end; cleared anyway in case that launch stopped early)
__global__ void clear_used_items(const Ctrl *ctrl, Item *items, int64_t cap) {
    const uint64_t r = ctrl->dq_reserve;
    const int64_t used = (int64_t)(r < (uint64_t)cap ? r : (uint64_t)cap);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t k = t; k < used; k += (int64_t)gridDim.x * blockDim.x) items[k].ready = 0u;
}

__global__ void clear_items(Item *items, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t k = t; k < n; k += (int64_t)gridDim.x * blockDim.x) items[k].ready = 0u;
}

// integer VALU probe: 8 independent and/or/xor/add chains per lane
__global__ void __launch_bounds__(256) valu_probe(int iters, uint32_t *sink) {
    uint32_t a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = threadIdx.x * 2654435761u + k;
    const uint32_t m = blockIdx.x | 1u;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = (a[k] ^ m) + 0x9E3779B9u;
            a[k] = (a[k] | (m << 3)) & 0xFFFF7FFFu;
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r ^= a[k];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int N, bool VS>
static hipError_t launch_n(const LaunchArgs &a) {
    const int block = a.block;
    const size_t lds = lds_bytes(N, a.plan.nlev, block);
    if (a.persistent) {
        const int grid = a.grid;
        hipLaunchKernelGGL(clear_used_items, dim3(256), dim3(256), 0, a.stream, a.ctrl, a.items, a.item_cap);
        hipLaunchKernelGGL(reset_ctrl, dim3(1024), dim3(256), 0, a.stream, a.ctrl, (uint64_t)a.num, a.counts,
                           a.num, a.status);
        if (a.steps)
            hipLaunchKernelGGL((persistent_kernel<N, VS, true>), dim3(grid), dim3(block), lds, a.stream, a.plan,
                               a.prefixes, a.num, a.counts, a.status, a.steps, a.ctrl, a.items, a.item_cap,
                               a.tune);
        else
            hipLaunchKernelGGL((persistent_kernel<N, VS, false>), dim3(grid), dim3(block), lds, a.stream, a.plan,
                               a.prefixes, a.num, a.counts, a.status, a.steps, a.ctrl, a.items, a.item_cap,
                               a.tune);
    } else {
        const int64_t grid = (a.num + block - 1) / block;
        if (a.steps)
            hipLaunchKernelGGL((plain_kernel<N, VS, true>), dim3((unsigned)grid), dim3(block), lds, a.stream, a.plan,
                               a.prefixes, a.num, a.counts, a.status, a.steps);
        else
            hipLaunchKernelGGL((plain_kernel<N, VS, false>), dim3((unsigned)grid), dim3(block), lds, a.stream,
                               a.plan, a.prefixes, a.num, a.counts, a.status, a.steps);
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_vs(const LaunchArgs &a) {
    return a.vs ? launch_n<N, true>(a) : launch_n<N, false>(a);
}

hipError_t launch(const LaunchArgs &a) {
    switch (a.n) {
        case 1: return launch_vs<1>(a);
        case 2: return launch_vs<2>(a);
        case 3: return launch_vs<3>(a);
        case 4: return launch_vs<4>(a);
        case 5: return launch_vs<5>(a);
        case 6: return launch_vs<6>(a);
        case 7: return launch_vs<7>(a);
        case 8: return launch_vs<8>(a);
        case 9: return launch_vs<9>(a);
        case 10: return launch_vs<10>(a);
        case 11: return launch_vs<11>(a);
        case 12: return launch_vs<12>(a);
        case 13: return launch_vs<13>(a);
        case 14: return launch_vs<14>(a);
        case 15: return launch_vs<15>(a);
        case 16: return launch_vs<16>(a);
        default: return hipErrorInvalidValue;
    }
}

uint32_t make_desc(int n, int i, int j) {
    const int lpw = 32 / n;
    uint32_t d = (uint32_t)((i % lpw) * n) | (uint32_t)(i / lpw) << 5 | (uint32_t)((j % lpw) * n) << 8 |
                 (uint32_t)(j / lpw) << 13;
    if (i == j) d |= 1u << 16;
    if (i + j == n - 1) d |= 1u << 17;
    return d;
}

size_t lds_bytes(int n, int nlev, int block) {
    const size_t elem = n <= 8 ? 1 : 2;
    return sizeof(uint32_t) * kMaxLevels + elem * (size_t)(nlev > 1 ? nlev : 1) * block;
}

hipError_t clear_item_flags(Item *items, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(clear_items, dim3(1024), dim3(256), 0, stream, items, n);
    return hipGetLastError();
}

hipError_t launch_valu_probe(int blocks, int iters, uint32_t *sink, hipStream_t stream) {
    hipLaunchKernelGGL(valu_probe, dim3(blocks), dim3(256), 0, stream, iters, sink);
    return hipGetLastError();
}

}  // namespace dlsk
