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
//  * the 2N+2 line masks live in VGPRs: row and column lines are N-bit fields
//    packed floor(64/N) to a 64-bit word (all eight lines of one kind in one
//    word up to N = 8); a per-level descriptor gives the bit offset of the
//    cell's row and column field, so reading a line is one 64-bit shift and
//    marking a value is one shift and an XOR;
//  * the per-lane stack holds, per level, the candidate set at the time the
//    level was left downwards (the taken value is its lowest bit); it lives
//    in LDS, one row per level with the lanes of a workgroup side by side;
//  * a DFS step is one instruction stream for every lane: go down one level
//    (take the lowest candidate) or up one level (clear the value taken there
//    and resume with the rest).  Marking and clearing are both XOR, so lanes
//    at different depths stay converged;
//  * a prep kernel turns each prefix (n*n cells) into a task record: packed
//    masks, level and candidate set.  The search kernels start tasks from
//    records, and a lane that gives away part of its tree writes the same
//    record (its masks rewound to the donated level).
//
// Vertical symmetry (Sec. 5.4): only the left half is searched; placing v at
// (i,j) also places N-1-v at (i,N-1-j).  Row masks receive both values,
// column masks are kept for the left half only (the right half mirrors them),
// and a value on one diagonal puts its mirror on the other.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "dls_kernels.hpp"

namespace dlsk {

// ---------------------------------------------------------------------------
// geometry of the packed masks and task records
// ---------------------------------------------------------------------------

template <int N, bool VS>
struct Geo {
    static constexpr int LPW = 64 / N;                        // lines per 64-bit word
    static constexpr int NCOL = VS ? (N + 1) / 2 : N;         // column lines kept
    static constexpr int WR = (N + LPW - 1) / LPW;            // words of row lines
    static constexpr int WC = (NCOL + LPW - 1) / LPW;         // words of column lines
    static constexpr uint32_t ALL = (1u << N) - 1u;
};

template <int N, bool VS>
struct alignas(16) Rec {
    uint64_t R[Geo<N, VS>::WR];
    uint64_t C[Geo<N, VS>::WC];
    uint32_t diag;    // md | ad << 16
    uint32_t cl;      // cand | level << 16; level kNone: nothing to search
    uint32_t origin;  // index of the prefix this task belongs to
    uint32_t pad;
};
constexpr uint32_t kNone = 0xFFFFu;

template <int W>
__device__ __forceinline__ uint64_t pickw(const uint64_t (&x)[W], uint32_t w) {
    uint64_t r = x[0];
#pragma unroll
    for (int k = 1; k < W; ++k) r = (w == (uint32_t)k) ? x[k] : r;
    return r;
}

template <int W>
__device__ __forceinline__ void flipw(uint64_t (&x)[W], uint32_t w, uint64_t bits) {
    if constexpr (W == 1) {
        x[0] ^= bits;
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k) x[k] ^= (w == (uint32_t)k) ? bits : 0ull;
    }
}

// LDS accesses through 32-bit LDS addresses (no generic-pointer arithmetic
// in the search loop)
template <class T>
__device__ __forceinline__ T lds_ld(uint32_t a) {
    return *reinterpret_cast<const __attribute__((address_space(3))) T *>((uintptr_t)a);
}
template <class T>
__device__ __forceinline__ void lds_st(uint32_t a, T v) {
    *reinterpret_cast<__attribute__((address_space(3))) T *>((uintptr_t)a) = v;
}
// 8-byte LDS load (one ds_read_b64)
__device__ __forceinline__ uint2 lds_ld2(uint32_t a) {
    typedef uint32_t v2u __attribute__((ext_vector_type(2)));
    const v2u v = *reinterpret_cast<const __attribute__((address_space(3))) v2u *>((uintptr_t)a);
    return make_uint2(v.x, v.y);
}
// 16-byte LDS load (one ds_read_b128)
__device__ __forceinline__ uint4 lds_ld4(uint32_t a) {
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const v4u v = *reinterpret_cast<const __attribute__((address_space(3))) v4u *>((uintptr_t)a);
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <class T>
__device__ __forceinline__ void lds_xor(uint32_t a, T v) {
    __hip_atomic_fetch_xor(reinterpret_cast<__attribute__((address_space(3))) T *>((uintptr_t)a), v,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// LDS address of a __shared__ object
__device__ __forceinline__ uint32_t lds_of(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

__device__ __forceinline__ uint32_t d_rw(uint32_t d) { return (d >> 6) & 3u; }
__device__ __forceinline__ uint32_t d_cw(uint32_t d) { return (d >> 14) & 3u; }
__device__ __forceinline__ uint32_t d_md(uint32_t d) { return 0u - ((d >> 16) & 1u); }
__device__ __forceinline__ uint32_t d_ad(uint32_t d) { return 0u - ((d >> 17) & 1u); }

template <int N, bool VS>
struct Lane {
    using G = Geo<N, VS>;
    uint64_t R[G::WR];  // row lines
    uint64_t C[G::WC];  // column lines (left half only with VS)
    uint32_t md, ad;    // diagonal masks
    uint32_t cand;      // remaining candidates at the current level
    uint32_t cur;       // descriptor of the current level's cell
    uint32_t da;        // LDS address of the current level's descriptor (base + 4 * level)
    uint32_t da0;       // the same for the level at which this task began
    uint32_t sa;        // LDS address of this lane's stack entry for the current level
    uint32_t c32;       // squares completed since the last flush()
    uint64_t cnt;       // squares completed by this task (after flush())

    // levels, given the LDS address of the descriptor table
    __device__ __forceinline__ int depth(uint32_t dbase) const { return (int)((da - dbase) >> 2); }
    __device__ __forceinline__ int start_level(uint32_t dbase) const { return (int)((da0 - dbase) >> 2); }
    __device__ __forceinline__ void flush() {
        cnt += c32;
        c32 = 0u;
    }

    __device__ __forceinline__ uint32_t cands(uint32_t desc) const {
        const uint32_t r = (uint32_t)(pickw<G::WR>(R, d_rw(desc)) >> (desc & 63u));
        const uint32_t c = (uint32_t)(pickw<G::WC>(C, d_cw(desc)) >> ((desc >> 8) & 63u));
        return G::ALL & ~(r | c | (md & d_md(desc)) | (ad & d_ad(desc)));
    }

    // mark or clear (XOR) the value bit b at the cell of `desc`
    __device__ __forceinline__ void toggle(uint32_t desc, uint32_t b) {
        const uint32_t mdm = d_md(desc), adm = d_ad(desc);
        if constexpr (VS) {
            const uint32_t rb = (1u << (N - 1)) >> (__builtin_ctz(b) & 31u);  // N-1-v
            flipw<G::WR>(R, d_rw(desc), (uint64_t)(b | rb) << (desc & 63u));
            flipw<G::WC>(C, d_cw(desc), (uint64_t)b << ((desc >> 8) & 63u));
            md ^= (b & mdm) | (rb & adm);
            ad ^= (b & adm) | (rb & mdm);
        } else {
            flipw<G::WR>(R, d_rw(desc), (uint64_t)b << (desc & 63u));
            flipw<G::WC>(C, d_cw(desc), (uint64_t)b << ((desc >> 8) & 63u));
            md ^= b & mdm;
            ad ^= b & adm;
        }
    }

    __device__ __forceinline__ bool done() const { return cand == 0u && da == da0; }

    // One DFS step.  Level descriptors sit 4 bytes apart and this lane's
    // stack entries `stride` bytes apart in LDS; da and sa track the current
    // level's entries, so moving one level is an add.  da_last = address of
    // the last level's descriptor.  Requires !done().
    template <class S>
    __device__ __forceinline__ void step(uint32_t stride, uint32_t da_last) {
        const bool up = (cand == 0u);
        const uint32_t nda = da + (up ? 0u - 4u : 4u);
        const uint32_t nsa = sa + (up ? 0u - stride : stride);
        const uint32_t ndesc = lds_ld<uint32_t>(nda);
        const uint32_t saved = lds_ld<S>(up ? nsa : sa);
        // up lanes write 0 into a slot nobody reads again
        lds_st<S>(sa, (S)cand);
        const uint32_t stored = up ? saved : cand;
        const uint32_t b = stored & (0u - stored);
        toggle(up ? ndesc : cur, b);
        const uint32_t nc = cands(ndesc);
        const bool leaf = (nda == da_last);
        c32 += leaf ? (uint32_t)__builtin_popcount(nc) : 0u;
        cand = up ? (stored ^ b) : (leaf ? 0u : nc);
        cur = ndesc;
        da = nda;
        sa = nsa;
    }

    // Start the task of record r.  dbase: LDS address of the descriptor
    // table; lane_off / stride: LDS address of this lane's level-0 stack entry
    // and the distance between levels.
    __device__ __forceinline__ void from_rec(const Rec<N, VS> &r, const uint32_t *sdesc, int last,
                                             uint32_t dbase = 0u, uint32_t lane_off = 0u, uint32_t stride = 0u) {
#pragma unroll
        for (int k = 0; k < G::WR; ++k) R[k] = r.R[k];
#pragma unroll
        for (int k = 0; k < G::WC; ++k) C[k] = r.C[k];
        md = r.diag & 0xFFFFu;
        ad = r.diag >> 16;
        cnt = 0;
        c32 = 0u;
        const uint32_t lvl = r.cl >> 16;
        if (lvl == kNone) {
            cand = 0u;
            da = da0 = dbase;
            sa = lane_off;
            return;
        }
        cand = r.cl & 0xFFFFu;
        da = da0 = dbase + 4u * lvl;
        sa = lane_off + lvl * stride;
        cur = sdesc[lvl];
        if ((int)lvl == last) {
            c32 = (uint32_t)__builtin_popcount(cand);
            cand = 0u;
        }
    }
};

// stack element: 8 bits suffice up to N = 8
template <int N>
using StackT = typename std::conditional<(N <= 8), uint8_t, uint16_t>::type;

// LDS layout of the plain kernel: 4-byte level descriptors, then the stacks
// (the persistent kernel's layouts follow LdsLane and VLane below)
constexpr uint32_t kStackBase = sizeof(uint32_t) * kMaxLevels;
// from this order on, the LDS-mask layout packs a row and a column mask into
// one word (see LdsLane)
constexpr int kLmPackMinN = 9;

// LDS layout with the line masks in LDS (LdsLane): a table of level
// descriptors (8 bytes each, 16 with VS; one per level of the plan), then the
// row and column masks (one 32-bit word per line and lane, lines apart by
// `lstride` = 4 * block bytes, lanes side by side), then the stacks.  LDS per
// lane sets the occupancy of this layout, so nothing is sized for the maximum.
__host__ __device__ inline uint32_t lm_desc_bytes(int nlev, bool vs) {
    return ((vs ? 16u : 8u) * (uint32_t)(nlev > 1 ? nlev : 1) + 15u) & ~15u;
}

__host__ __device__ inline uint32_t lm_stack_base(int lines, int nlev, int block, bool vs) {
    return lm_desc_bytes(nlev, vs) + 4u * (uint32_t)lines * (uint32_t)block;
}

__host__ __device__ inline uint32_t lm_stacks_end(int lines, int nlev, int block, int elem, bool vs) {
    const uint32_t end =
        lm_stack_base(lines, nlev, block, vs) + (uint32_t)elem * (uint32_t)(nlev > 1 ? nlev : 1) * (uint32_t)block;
    return (end + 15u) & ~15u;
}

// Lane state with the row and column masks in LDS instead of VGPRs.  A value
// is marked or cleared with one LDS xor per line (ds_xor_b32), so the packed
// 64-bit words and their word selection disappear from the search loop;
// only the diagonal masks stay in registers.  A level descriptor holds the
// LDS offsets of the cell's row and column mask words and the diagonal
// selectors as all-ones / zero masks (layouts below).
template <int N, bool VS>
struct LdsLane {
    using G = Geo<N, VS>;
    // PACK: LDS word k of a lane holds row k's mask in bits 0-15 and column
    // k's mask in bits 16-31 (half the LDS, one shift more per toggle and
    // read); otherwise one word per row, then one per column
    static constexpr bool PACK = N >= kLmPackMinN;
    static constexpr int LINES = PACK ? N : N + G::NCOL;
    static constexpr uint32_t CSH = PACK ? 16u : 0u;  // column mask position in its word
    // Level descriptors: 8 bytes {row word offset | column word offset << 16,
    // main-diagonal selector | antidiagonal selector << 16}, the current
    // level's kept in registers; with VS 16 bytes {row offset, column offset,
    // main selector, anti selector}, both read from LDS at each step (the
    // 8-byte form measured 15 % slower on the vertically symmetric order-10
    // count and 7 % faster on order 9)
    static constexpr uint32_t DB = VS ? 16u : 8u;
    static constexpr uint32_t DSH = VS ? 4u : 3u;
    uint32_t md;        // main-diagonal mask
    uint32_t ad2;       // antidiagonal mask (VS) or antidiagonal mask << 16
    uint32_t cand;      // remaining candidates at the current level
    uint2 cur;          // descriptor of the current level's cell (not VS)
    uint32_t da;        // LDS address of the current level's descriptor (base + DB * level)
    uint32_t da0;       // the same for the level at which this task began
    uint32_t sa;        // LDS address of this lane's stack entry for the current level
    uint32_t mbase;     // LDS address of this lane's row-0 mask word
    uint32_t c32;       // squares completed since the last flush()
    uint64_t cnt;       // squares completed by this task (after flush())

    __device__ __forceinline__ int depth(uint32_t dbase) const { return (int)((da - dbase) >> DSH); }
    __device__ __forceinline__ int start_level(uint32_t dbase) const { return (int)((da0 - dbase) >> DSH); }
    __device__ __forceinline__ void flush() {
        cnt += c32;
        c32 = 0u;
    }
    __device__ __forceinline__ bool done() const { return cand == 0u && da == da0; }

    // mark or clear the value bit b at the cell of an 8-byte descriptor t
    // (not VS); dmd / dadh are the diagonal masks to update
    __device__ __forceinline__ void toggle_at(const uint2 &t, uint32_t b, uint32_t &dmd, uint32_t &dadh) const {
        lds_xor(mbase + (t.x & 0xFFFFu), b);
        lds_xor(mbase + (t.x >> 16), b << CSH);
        dmd ^= b & t.y;
        dadh ^= (b << 16) & t.y;
    }
    // the same for a 16-byte descriptor (VS: the mirrored value N-1-v is
    // marked in the same row, and the diagonals swap for it)
    __device__ __forceinline__ void toggle_at(const uint4 &t, uint32_t b, uint32_t &dmd, uint32_t &dad) const {
        const uint32_t rb = (1u << (N - 1)) >> (__builtin_ctz(b) & 31u);  // N-1-v
        lds_xor(mbase + t.x, b | rb);
        lds_xor(mbase + t.y, b << CSH);
        dmd ^= (b & t.z) | (rb & t.w);
        dad ^= (b & t.w) | (rb & t.z);
    }
    // toggle at level l's cell, descriptor read from LDS
    __device__ __forceinline__ void toggle_level(uint32_t dbase, int l, uint32_t b, uint32_t &dmd, uint32_t &dad) const {
        if constexpr (VS) toggle_at(lds_ld4(dbase + DB * (uint32_t)l), b, dmd, dad);
        else toggle_at(lds_ld2(dbase + DB * (uint32_t)l), b, dmd, dad);
    }

    // One DFS step, taken by every lane of the wave, busy or not.  A lane
    // without work (its task finished, or none yet) sits at its start level
    // with no candidates, and its up move is clamped there.  The first such
    // step XORs the start slot's stale bit into the lane's own masks (the
    // next task's from_rec() overwrites them) and writes 0 into that slot;
    // from then on the step changes nothing.  So the search loop needs no
    // per-lane test and no exec-mask merges.
    // The new stack address follows from the new descriptor address:
    // nsa = nda * kst + sc0 (kst = stride / DB, sc0 = stack address of
    // level 0 minus dbase * kst, modulo 2^32).
    template <class S>
    __device__ __forceinline__ void step(uint32_t kst, uint32_t sc0, uint32_t da_last) {
        const bool up = (cand == 0u);
        const uint32_t nda = (uint32_t)max((int)(da + (up ? 0u - DB : DB)), (int)da0);
        const uint32_t nsa = __umul24(nda, kst) + sc0;
        uint32_t nc, stored, b;
        if constexpr (VS) {
            const uint4 nd = lds_ld4(nda);
            const uint4 td = lds_ld4(up ? nda : da);  // the cell whose value is marked or cleared
            const uint32_t saved = lds_ld<S>(up ? nsa : sa);
            lds_st<S>(sa, (S)cand);  // up lanes write 0 into a slot nobody reads again
            stored = up ? saved : cand;
            b = stored & (0u - stored);
            toggle_at(td, b, md, ad2);
            const uint32_t r = lds_ld<uint32_t>(mbase + nd.x), c = lds_ld<uint32_t>(mbase + nd.y) >> CSH;
            nc = G::ALL & ~(r | c | (md & nd.z) | (ad2 & nd.w));
        } else {
            const uint2 nd = lds_ld2(nda);
            const uint32_t saved = lds_ld<S>(up ? nsa : sa);
            lds_st<S>(sa, (S)cand);  // up lanes write 0 into a slot nobody reads again
            stored = up ? saved : cand;
            b = stored & (0u - stored);
            toggle_at(up ? nd : cur, b, md, ad2);  // the cell whose value is marked or cleared
            // PACK: the row word's upper half (a column mask) falls outside ALL
            const uint32_t r = lds_ld<uint32_t>(mbase + (nd.x & 0xFFFFu));
            const uint32_t c = lds_ld<uint32_t>(mbase + (nd.x >> 16)) >> CSH;
            nc = G::ALL & ~(r | c | (md & nd.y) | ((ad2 & nd.y) >> 16));
            cur = nd;
        }
        const bool leaf = (nda == da_last) && !up;
        c32 += leaf ? (uint32_t)__builtin_popcount(nc) : 0u;
        cand = up ? (stored ^ b) : (leaf ? 0u : nc);
        da = nda;
        sa = nsa;
    }

    // Start the task of record r: its masks go to this lane's LDS words.
    __device__ __forceinline__ void from_rec(const Rec<N, VS> &r, uint32_t dbase, int last, uint32_t lane_off,
                                             uint32_t stride, uint32_t lstride) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            uint32_t w = (uint32_t)(r.R[i / G::LPW] >> ((i % G::LPW) * N)) & G::ALL;
            if (PACK && i < G::NCOL) w |= ((uint32_t)(r.C[i / G::LPW] >> ((i % G::LPW) * N)) & G::ALL) << 16;
            lds_st<uint32_t>(mbase + (uint32_t)i * lstride, w);
        }
        if constexpr (!PACK) {
#pragma unroll
            for (int j = 0; j < G::NCOL; ++j)
                lds_st<uint32_t>(mbase + (uint32_t)(N + j) * lstride,
                                 (uint32_t)(r.C[j / G::LPW] >> ((j % G::LPW) * N)) & G::ALL);
        }
        md = r.diag & 0xFFFFu;
        ad2 = VS ? r.diag >> 16 : r.diag & 0xFFFF0000u;
        cnt = 0;
        c32 = 0u;
        const uint32_t lvl = r.cl >> 16;
        if (lvl == kNone) {
            cand = 0u;
            da = da0 = dbase;
            sa = lane_off;
            if constexpr (!VS) cur = lds_ld2(dbase);
            return;
        }
        cand = r.cl & 0xFFFFu;
        da = da0 = dbase + DB * lvl;
        sa = lane_off + lvl * stride;
        if constexpr (!VS) cur = lds_ld2(da);
        if ((int)lvl == last) {
            c32 = (uint32_t)__builtin_popcount(cand);
            cand = 0u;
        }
    }

    // Give away the untried siblings at level lvl (see donate()): the masks
    // are rewound in place to lvl, copied into the record, then replayed.
    template <class SlotOf>
    __device__ __forceinline__ Rec<N, VS> donate(int lvl, uint32_t dbase, SlotOf slot_of, uint32_t origin,
                                                 uint32_t lstride) const {
        const int dep = depth(dbase);
        uint32_t tmd = md, tad = ad2;
        for (int l = dep - 1; l >= lvl; --l) {
            const uint32_t sv = *slot_of(l);
            toggle_level(dbase, l, sv & (0u - sv), tmd, tad);
        }
        Rec<N, VS> r;
#pragma unroll
        for (int k = 0; k < G::WR; ++k) r.R[k] = 0;
#pragma unroll
        for (int k = 0; k < G::WC; ++k) r.C[k] = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const uint32_t w = lds_ld<uint32_t>(mbase + (uint32_t)i * lstride);
            r.R[i / G::LPW] |= (uint64_t)(w & 0xFFFFu) << ((i % G::LPW) * N);
            if (PACK && i < G::NCOL) r.C[i / G::LPW] |= (uint64_t)(w >> 16) << ((i % G::LPW) * N);
        }
        if constexpr (!PACK) {
#pragma unroll
            for (int j = 0; j < G::NCOL; ++j)
                r.C[j / G::LPW] |= (uint64_t)lds_ld<uint32_t>(mbase + (uint32_t)(N + j) * lstride)
                                   << ((j % G::LPW) * N);
        }
        uint32_t rmd = tmd, rad = tad;
        for (int l = lvl; l < dep; ++l) {  // replay: this lane keeps its branch
            const uint32_t sv = *slot_of(l);
            toggle_level(dbase, l, sv & (0u - sv), rmd, rad);
        }
        const uint32_t sv = *slot_of(lvl);
        const uint32_t b = sv & (0u - sv);
        r.diag = tmd | (VS ? tad << 16 : tad);
        r.cl = (sv ^ b) | ((uint32_t)lvl << 16);
        r.origin = origin;
        r.pad = 0;
        *slot_of(lvl) = (decltype(*slot_of(lvl) + 0))b;
        return r;
    }
};

// Lane state of the persistent kernel with the line masks in VGPRs (packed
// 64-bit words as in Lane) and level descriptors in LDS.
//
// Even N <= 8 without vertical symmetry (no cell lies on both diagonals;
// one 64-bit word per kind of line): 16-byte descriptors {row shift, column
// shift, diagonal shift, leaf increment}.  Both diagonal masks live in one
// word D: main diagonal in bits 0-7, antidiagonal in bits 8-15, bits 16-23
// zero and bits 24-31 all ones.  The diagonal shift is 0 or 8 for a cell on
// the main or the antidiagonal, 48 for a cell on neither: marking uses the
// low word of a 64-bit shift (nothing, for 48), reading a 32-bit shift,
// which takes the shift modulo 32 (the zero field, for 48).  One level past
// the last (the sentinel) has shift 56: nothing to mark, and it reads the
// all-ones field, so a lane that steps onto it has no candidates and goes
// back up; its increment is 1, so every square is counted by the step that
// reaches the sentinel (two extra steps per square instead of a popcount and
// a leaf test in every step).
//
// Otherwise: 8-byte descriptors
//   x = row shift | row word << 6 | (on main diagonal ? ALL << 16 : 0)
//   y = column shift | column word << 6 | keep << 8 | (on antidiagonal ? ALL << 16 : 0)
// The 64-bit shifts read only the low 6 bits of x / y, and the diagonal
// masks are kept in bits 16-31 (mdh, adh), so a diagonal test is one AND
// with x or y: no field extraction in the search loop.  keep (N <= 8):
// AllN, and 0 at the last level, whose candidates are counted instead of
// entered.
constexpr uint32_t kVlStackBase = 8u * kMaxLevels;

__host__ __device__ inline uint32_t vl_stacks_end(int nlev, int block, int elem) {
    const uint32_t end = kVlStackBase + (uint32_t)elem * (uint32_t)(nlev > 1 ? nlev : 1) * (uint32_t)block;
    return (end + 15u) & ~15u;
}

// diagonal shifts of the D form
constexpr uint32_t kDwNone = 48u;      // on neither diagonal
constexpr uint32_t kDwSentinel = 56u;  // the level past the last

template <int N, bool VS>
struct VLaneDesc {
    // D word form: even order, no vertical symmetry, 8-bit lines
    static constexpr bool DW = (N % 2 == 0) && !VS && N <= 8;
    static constexpr uint32_t DB = DW ? 16u : 8u;      // descriptor bytes
    static constexpr uint32_t DSH = DW ? 4u : 3u;
    using T = typename std::conditional<DW, uint4, uint2>::type;
    // stack rows and descriptors a plan of nlev levels needs (D form: one
    // more, the sentinel)
    __host__ __device__ static int rows(int nlev) { return DW ? nlev + 1 : nlev; }
    __device__ __forceinline__ static T load(uint32_t a) {
        if constexpr (DW) return lds_ld4(a);
        else return lds_ld2(a);
    }
};
// the 16-byte descriptor table spans 128 levels, more than any order <= 8 has
static_assert(16u * 128u <= kVlStackBase, "descriptor table overlaps the stacks");

template <int N, bool VS>
struct VLane {
    using G = Geo<N, VS>;
    using DT = VLaneDesc<N, VS>;
    using Desc = typename DT::T;
    static constexpr bool DW = DT::DW;
    static constexpr uint32_t DB = DT::DB;
    uint64_t R[G::WR];  // row lines
    uint64_t C[G::WC];  // column lines (left half only with VS)
    uint32_t mdh, adh;  // diagonal masks << 16 (D form: the word D in mdh)
    uint32_t cand;      // remaining candidates at the current level
    Desc cur;           // descriptor of the current level's cell
    uint32_t da;        // LDS address of the current level's descriptor (base + DB * level)
    uint32_t da0;       // the same for the level at which this task began
    uint32_t sa;        // LDS address of this lane's stack entry for the current level
    uint32_t c32;       // squares completed since the last flush()
    uint64_t cnt;       // squares completed by this task (after flush())

    __device__ __forceinline__ int depth(uint32_t dbase) const { return (int)((da - dbase) >> DT::DSH); }
    __device__ __forceinline__ int start_level(uint32_t dbase) const { return (int)((da0 - dbase) >> DT::DSH); }
    __device__ __forceinline__ void flush() {
        cnt += c32;
        c32 = 0u;
    }
    __device__ __forceinline__ bool done() const { return cand == 0u && da == da0; }

    // all lines of the cell of d: row | column | diagonals (bits above N undefined)
    __device__ __forceinline__ uint32_t lines(const Desc &d) const {
        if constexpr (DW) {
            return (uint32_t)(R[0] >> d.x) | (uint32_t)(C[0] >> d.y) | (mdh >> (d.z & 31u));
        } else {
            const uint32_t r = (uint32_t)(pickw<G::WR>(R, (d.x >> 6) & 3u) >> (d.x & 63u));
            const uint32_t c = (uint32_t)(pickw<G::WC>(C, (d.y >> 6) & 3u) >> (d.y & 63u));
            return r | c | (((mdh & d.x) | (adh & d.y)) >> 16);
        }
    }
    __device__ __forceinline__ uint32_t cands(const Desc &d) const { return G::ALL & ~lines(d); }

    // mark or clear (XOR) the value bit b at the cell of descriptor d
    __device__ __forceinline__ void toggle(const Desc &d, uint32_t b) {
        if constexpr (DW) {
            R[0] ^= (uint64_t)b << d.x;
            C[0] ^= (uint64_t)b << d.y;
            mdh ^= (uint32_t)((uint64_t)b << d.z);  // nothing for a shift >= 32
        } else {
            const uint32_t bh = b << 16;
            if constexpr (VS) {
                const uint32_t rb = (1u << (N - 1)) >> (__builtin_ctz(b) & 31u);  // N-1-v
                const uint32_t rbh = rb << 16;
                flipw<G::WR>(R, (d.x >> 6) & 3u, (uint64_t)(b | rb) << (d.x & 63u));
                flipw<G::WC>(C, (d.y >> 6) & 3u, (uint64_t)b << (d.y & 63u));
                mdh ^= (bh & d.x) | (rbh & d.y);
                adh ^= (bh & d.y) | (rbh & d.x);
            } else {
                flipw<G::WR>(R, (d.x >> 6) & 3u, (uint64_t)b << (d.x & 63u));
                flipw<G::WC>(C, (d.y >> 6) & 3u, (uint64_t)b << (d.y & 63u));
                mdh ^= bh & d.x;
                adh ^= bh & d.y;
            }
        }
    }

    // One DFS step, taken by every lane of the wave (see LdsLane::step for
    // the parked lanes).  nsa = nda * kst + sc0 (kst = stride / DB).  Up to
    // N = 8 a keep mask is AllN, and 0 at the last level, whose candidates
    // are counted instead of entered; no lane is ever parked at the last
    // level (see from_rec), so an up step never lands on it and needs no
    // guard.  The stack read at nsa serves up lanes (the slot they return
    // to); a down lane reads the slot below it, which it does not use.
    template <class S>
    __device__ __forceinline__ void step(uint32_t kst, uint32_t sc0, uint32_t da_last) {
        const bool up = (cand == 0u);
        const uint32_t nda = (uint32_t)max((int)(da + (up ? 0u - DB : DB)), (int)da0);
        const uint32_t nsa = __umul24(nda, kst) + sc0;
        const Desc nd = DT::load(nda);
        // the descriptor of the level whose value changes (the new level
        // going up, the current one going down): one more LDS read instead
        // of selecting its fields in registers
        const Desc td = DT::load(up ? nda : da);
        const uint32_t saved = lds_ld<S>(nsa);
        lds_st<S>(sa, (S)cand);  // up lanes write 0 into a slot nobody reads again
        const uint32_t stored = up ? saved : cand;
        const uint32_t b = stored & (0u - stored);
        toggle(td, b);
        if constexpr (DW) {
            // a square is counted on reaching the sentinel (increment 1);
            // both candidate sets are formed and one is kept by a mask, so
            // the step stays one branch-free instruction stream
            c32 += nd.w;
            const uint32_t upm = 0u - (uint32_t)up;
            cand = ((stored ^ b) & upm) | (G::ALL & ~lines(nd) & ~upm);
        } else {
            const uint32_t nc = cands(nd);
            if constexpr (N <= 8) {
                const uint32_t keep = (nd.y >> 8) & 0xFFu;
                c32 += (uint32_t)__builtin_popcount(nc & ~keep);
                cand = up ? (stored ^ b) : (nc & keep);
            } else {
                const bool leaf = (nda == da_last) && !up;
                c32 += leaf ? (uint32_t)__builtin_popcount(nc) : 0u;
                cand = up ? (stored ^ b) : (leaf ? 0u : nc);
            }
        }
        da = nda;
        sa = nsa;
    }

    // Start the task of record r (dbase: LDS address of the descriptor
    // table; lane_off / stride: this lane's level-0 stack entry and the
    // distance between levels).
    __device__ __forceinline__ void from_rec(const Rec<N, VS> &r, uint32_t dbase, int last, uint32_t lane_off,
                                             uint32_t stride) {
#pragma unroll
        for (int k = 0; k < G::WR; ++k) R[k] = r.R[k];
#pragma unroll
        for (int k = 0; k < G::WC; ++k) C[k] = r.C[k];
        if constexpr (DW) {
            mdh = (r.diag & 0xFFu) | ((r.diag >> 8) & 0xFF00u) | (G::ALL << 24);
            adh = 0u;
        } else {
            mdh = r.diag << 16;
            adh = r.diag & 0xFFFF0000u;
        }
        cnt = 0;
        c32 = 0u;
        const uint32_t lvl = r.cl >> 16;
        if (lvl == kNone) {
            cand = 0u;
            da = da0 = dbase;
            sa = lane_off;
            cur = DT::load(dbase);
            return;
        }
        cand = r.cl & 0xFFFFu;
        uint32_t at = lvl;
        if ((int)lvl == last) {
            c32 = (uint32_t)__builtin_popcount(cand);
            cand = 0u;
            at = lvl - 1u;  // parked one level up (the plan has at least two levels)
        }
        da = da0 = dbase + DB * at;
        sa = lane_off + at * stride;
        cur = DT::load(da);
    }

    // Give away the untried siblings at level lvl: the record holds the
    // masks as they were on entering lvl (the values taken at levels
    // lvl..depth-1 cleared again) and the candidates not yet tried there;
    // the lane keeps only the branch in progress.
    template <class SlotOf>
    __device__ __forceinline__ Rec<N, VS> donate(int lvl, uint32_t dbase, SlotOf slot_of, uint32_t origin) const {
        VLane T = *this;
        for (int l = depth(dbase) - 1; l >= lvl; --l) {
            const uint32_t sv = *slot_of(l);
            T.toggle(DT::load(dbase + DB * (uint32_t)l), sv & (0u - sv));
        }
        const uint32_t sv = *slot_of(lvl);
        const uint32_t b = sv & (0u - sv);
        Rec<N, VS> r;
#pragma unroll
        for (int k = 0; k < G::WR; ++k) r.R[k] = T.R[k];
#pragma unroll
        for (int k = 0; k < G::WC; ++k) r.C[k] = T.C[k];
        if constexpr (DW) r.diag = (T.mdh & 0xFFu) | ((T.mdh & 0xFF00u) << 8);
        else r.diag = (T.mdh >> 16) | (T.adh & 0xFFFF0000u);
        r.cl = (sv ^ b) | ((uint32_t)lvl << 16);
        r.origin = origin;
        r.pad = 0;
        *slot_of(lvl) = (decltype(*slot_of(lvl) + 0))b;
        return r;
    }
};

// descriptor table of VLane from the plan
template <int N, bool VS>
__device__ __forceinline__ void vl_build_desc(const Plan &plan, unsigned char *smem) {
    using G = Geo<N, VS>;
    for (int k = threadIdx.x; k < plan.nlev; k += blockDim.x) {
        const uint32_t d = plan.desc[k];
        // keep mask (N <= 8): AllN except at the last level
        const uint32_t keep = (N <= 8 && k != plan.nlev - 1) ? G::ALL : 0u;
        if constexpr (VLaneDesc<N, VS>::DW) {
            // one word per kind of line: the shifts are the bit offsets
            const uint32_t z = (d >> 16) & 1u ? 0u : ((d >> 17) & 1u ? 8u : kDwNone);
            reinterpret_cast<uint4 *>(smem)[k] = make_uint4(d & 63u, (d >> 8) & 63u, z, 0u);
        } else {
            reinterpret_cast<uint2 *>(smem)[k] =
                make_uint2((d & 0xFFu) | ((d_md(d) & G::ALL) << 16),
                           ((d >> 8) & 0xFFu) | (keep << 8) | ((d_ad(d) & G::ALL) << 16));
        }
    }
    if constexpr (VLaneDesc<N, VS>::DW) {
        if (threadIdx.x == 0) reinterpret_cast<uint4 *>(smem)[plan.nlev] = make_uint4(0u, 0u, kDwSentinel, 1u);
    }
}

// descriptor table of the LDS-mask layout from the plan (one entry per level)
template <int N, bool VS>
__device__ __forceinline__ void lm_build_desc(const Plan &plan, unsigned char *smem, uint32_t lstride) {
    using G = Geo<N, VS>;
    uint2 *t = reinterpret_cast<uint2 *>(smem);
    uint4 *t4 = reinterpret_cast<uint4 *>(smem);
    for (int k = threadIdx.x; k < plan.nlev; k += blockDim.x) {
        const uint32_t d = plan.desc[k];
        const uint32_t i = ((d >> 6) & 3u) * G::LPW + (d & 63u) / N;
        const uint32_t j = ((d >> 14) & 3u) * G::LPW + ((d >> 8) & 63u) / N;
        // word offsets fit 16 bits: at most (LINES - 1) * 4 * 1024 bytes
        static_assert((LdsLane<N, VS>::LINES - 1) * 4 * 1024 < 65536, "LDS-mask word offsets exceed 16 bits");
        const uint32_t roff = i * lstride, coff = (LdsLane<N, VS>::PACK ? j : N + j) * lstride;
        if constexpr (VS) t4[k] = make_uint4(roff, coff, d_md(d), d_ad(d));
        else t[k] = make_uint2(roff | (coff << 16), (d_md(d) & G::ALL) | ((d_ad(d) & G::ALL) << 16));
    }
}

// One prefix (cells in 32-bit words, four per word) -> its task record and
// the count it already determines (a dead, complete or one-level prefix).
// patbits: the cells every prefix of the plan assigns; desc0: the first
// level's 4-byte descriptor.  *mis: the prefix's assigned cells differ from
// the pattern (its count is then 0).
template <int N, bool VS>
__device__ __forceinline__ Rec<N, VS> prefix_record(const uint32_t *words, const uint32_t *patbits, uint32_t desc0,
                                                    int nlev, uint32_t origin, uint64_t *count, bool *mismatch) {
    using G = Geo<N, VS>;
    constexpr int NN = N * N;
    Lane<N, VS> L;
#pragma unroll
    for (int k = 0; k < G::WR; ++k) L.R[k] = 0;
#pragma unroll
    for (int k = 0; k < G::WC; ++k) L.C[k] = 0;
    L.md = L.ad = 0u;
    uint64_t bad = 0;
    uint32_t mis = 0u;
#pragma unroll
    for (int c = 0; c < NN; ++c) {
        const int i = c / N, j = c % N;
        const uint32_t v = (words[c >> 2] >> (8 * (c & 3))) & 0xFFu;
        const bool inpat = (patbits[c >> 5] >> (c & 31)) & 1u;
        const bool filled = v != 0xFFu;
        mis |= ((inpat != filled) || (filled && v >= (uint32_t)N)) ? 1u : 0u;
        if (!inpat || !filled || v >= (uint32_t)N) continue;
        const uint32_t b = 1u << v;
        const int rw = i / G::LPW, rs = (i % G::LPW) * N;
        if constexpr (VS) {
            if (2 * j > N - 1) continue;  // right half: taken care of through its mirror
            const int mc = i * N + (N - 1 - j);
            const uint32_t w = (words[mc >> 2] >> (8 * (mc & 3))) & 0xFFu;
            bad |= (w != (uint32_t)(N - 1) - v) ? 1u : 0u;
            // a cell on the middle column (odd N) is its own mirror: v = (N-1)/2
            const bool self = (2 * j == N - 1);
            if (self) bad |= (2 * v != (uint32_t)(N - 1)) ? 1u : 0u;
            const uint32_t rb = self ? 0u : 1u << (N - 1 - v);
            const int cw = j / G::LPW, cs = (j % G::LPW) * N;
            const uint64_t rbits = (uint64_t)(b | rb) << rs, cbits = (uint64_t)b << cs;
            bad |= (L.R[rw] & rbits) | (L.C[cw] & cbits);
            L.R[rw] |= rbits;
            L.C[cw] |= cbits;
            if (i == j) {
                bad |= (L.md & b) | (L.ad & rb);
                L.md |= b;
                L.ad |= rb;
            }
            if (i + j == N - 1) {
                bad |= (L.ad & b) | (L.md & rb);
                L.ad |= b;
                L.md |= rb;
            }
        } else {
            const int cw = j / G::LPW, cs = (j % G::LPW) * N;
            const uint64_t rbits = (uint64_t)b << rs, cbits = (uint64_t)b << cs;
            bad |= (L.R[rw] & rbits) | (L.C[cw] & cbits);
            L.R[rw] |= rbits;
            L.C[cw] |= cbits;
            if (i == j) {
                bad |= L.md & b;
                L.md |= b;
            }
            if (i + j == N - 1) {
                bad |= L.ad & b;
                L.ad |= b;
            }
        }
    }
    *mismatch = mis != 0u;
    Rec<N, VS> r;
#pragma unroll
    for (int k = 0; k < G::WR; ++k) r.R[k] = L.R[k];
#pragma unroll
    for (int k = 0; k < G::WC; ++k) r.C[k] = L.C[k];
    r.diag = L.md | (L.ad << 16);
    r.origin = origin;
    r.pad = 0;
    uint64_t cnt = 0;
    if (bad || mis) {
        r.cl = kNone << 16;
    } else if (nlev == 0) {
        cnt = 1;  // a complete, consistent square
        r.cl = kNone << 16;
    } else {
        const uint32_t c0 = L.cands(desc0);
        if (nlev == 1) {
            cnt = (uint64_t)__builtin_popcount(c0);
            r.cl = kNone << 16;
        } else {
            r.cl = c0;  // level 0
        }
    }
    *count = cnt;
    return r;
}

// ---------------------------------------------------------------------------
// prep: prefix cells -> task record (one lane per prefix)
// ---------------------------------------------------------------------------

template <int N, bool VS>
__global__ void __launch_bounds__(256) prep_kernel(const Plan plan, const uint8_t *__restrict__ prefixes,
                                                   int64_t num, Rec<N, VS> *__restrict__ recs,
                                                   uint64_t *__restrict__ counts, uint32_t *status) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= num) return;
    constexpr int NN = N * N;
    constexpr int NW = (NN + 3) / 4;
    const uint8_t *sq = prefixes + idx * NN;
    uint32_t words[NW];
    if constexpr (NN % 4 == 0) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(sq);
#pragma unroll
        for (int k = 0; k < NW; ++k) words[k] = w[k];
    } else {
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            uint32_t x = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * k + t < NN) x |= (uint32_t)sq[4 * k + t] << (8 * t);
            words[k] = x;
        }
    }
    uint64_t count = 0;
    bool mis = false;
    const Rec<N, VS> r = prefix_record<N, VS>(words, plan.patbits, plan.desc[0], plan.nlev, (uint32_t)idx, &count, &mis);
    if (mis && status) atomicOr(status, 1u);
    recs[idx] = r;
    counts[idx] = count;
}

// Byte offset of thread tid's stack slot within a level row of the
// search kernels' stacks (nthreads slots of `size` bytes).  With the
// lanes side by side, four lanes share each 4-byte word, and lanes at
// different levels meet in the same bank.  Instead the words are dealt out
// per lane: the slots of one wave's 64 lanes fall in 64 consecutive words --
// one per LDS bank, whatever level each lane is at -- and the threads sharing
// a word belong to different waves.  A row stays nthreads * size bytes when
// the waves fill the words (a multiple of 4 / size waves); otherwise the
// plain order is kept.
__device__ __forceinline__ uint32_t stack_slot(uint32_t tid, uint32_t nthreads, uint32_t size) {
    const uint32_t per = 4u / size;  // threads per word
    if ((nthreads >> 6) % per) return tid * size;
    const uint32_t wave = tid >> 6, lane = tid & 63u;
    return ((wave / per) * 64u + lane) * 4u + (wave % per) * size;
}

// ---------------------------------------------------------------------------
// plain kernel: one task per lane, run to completion
// ---------------------------------------------------------------------------

template <int N, bool VS, bool STATS>
__global__ void __launch_bounds__(1024) plain_kernel(const Plan plan, const Rec<N, VS> *__restrict__ recs,
                                                     int64_t num, uint64_t *__restrict__ counts,
                                                     uint64_t *steps) {
    using S = StackT<N>;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *sdesc = reinterpret_cast<uint32_t *>(smem);
    const int nlev = plan.nlev;
    for (int k = threadIdx.x; k < nlev; k += blockDim.x) sdesc[k] = plan.desc[k];
    __syncthreads();

    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t nsteps = 0;
    // a dead or complete prefix: result already written by the prep kernel
    const bool live = idx < num && (recs[idx < num ? idx : 0].cl >> 16) != kNone;
    if (live) {
        const Rec<N, VS> r = recs[idx];
        const uint32_t dbase = lds_of(smem);
        const uint32_t lane_off = dbase + kStackBase + stack_slot(threadIdx.x, blockDim.x, (uint32_t)sizeof(S));
        const uint32_t stride = blockDim.x * (uint32_t)sizeof(S);
        const uint32_t da_last = dbase + 4u * (uint32_t)(nlev - 1);
        Lane<N, VS> L;
        L.from_rec(r, sdesc, nlev - 1, dbase, lane_off, stride);
        // the 32-bit step counter is folded into the 64-bit count every 256 steps
        for (;;) {
            for (int k = 0; k < 256 && !L.done(); ++k) {
                L.template step<S>(stride, da_last);
                if (STATS) ++nsteps;
            }
            L.flush();
            if (L.done()) break;
        }
        counts[idx] = L.cnt;
    }
    if (STATS && steps) {
        if (live) atomicAdd((unsigned long long *)steps, (unsigned long long)nsteps);
        // a wave issues as many steps as its longest lane takes (every lane of
        // the wave takes part in the shuffles: none has returned)
        uint64_t wmax = nsteps;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t y = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(wmax >> 32), o) << 32) |
                               (uint32_t)__shfl_xor((int)(uint32_t)wmax, o);
            wmax = y > wmax ? y : wmax;
        }
        if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long *)(steps + 1), (unsigned long long)(wmax * 64u));
    }
}

// ---------------------------------------------------------------------------
// persistent kernel: global queue of tasks, lane-level refill, and donation
// of untried siblings when the static queue is exhausted
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lane index of the set bit of rank k in mask (k < popcount(mask)): the
// largest p with popcount(mask below p) <= k, by binary search
__device__ __forceinline__ int kth_lane(uint64_t mask, uint32_t k) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int p = pos + w;
        if ((uint32_t)__popcll(mask & ((1ull << p) - 1ull)) <= k) pos = p;
    }
    return pos;
}

// value of v in lane src, word by word (every lane of the wave must take part)
template <class T>
__device__ __forceinline__ T shfl_words(const T &v, int src) {
    static_assert(sizeof(T) % 4 == 0, "shuffled in 32-bit words");
    T out;
    const uint32_t *a = reinterpret_cast<const uint32_t *>(&v);
    uint32_t *o = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) o[k] = (uint32_t)__shfl((int)a[k], src, 64);
    return out;
}

__device__ __forceinline__ uint64_t bcast64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// s_memrealtime ticks at 100 MHz: 20 s without any queue progress ends the kernel
constexpr uint64_t kStallTicks = 100000000ull * 20;

// s_waitcnt immediate for gfx9: vmcnt = 0 (bits 3:0 and 15:14), no wait on
// expcnt (bits 6:4 = 7) or lgkmcnt (bits 11:8 = 15)
constexpr int kWaitVm0 = 0x0F70;

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x);

// The workgroup pool of the persistent kernel's tail (line masks in VGPRs):
// the record area after the stacks holds one record per thread; its first
// half is a 32-record mailbox per wave (sharing inside a wave), the second
// half the pool: a header (lock, record count, then idle and busy lanes of
// each of up to 16 waves) and the pooled records.
constexpr uint32_t kPoolHeader = 256u;
constexpr int kPoolIdle = 2, kPoolBusy = 18;  // word offsets in the header
constexpr uint32_t kMailbox = 32u;            // records per wave

// GL: donation across the chip compiled in (small batches); without it the
// kernel carries none of that code, which keeps its register use down.
template <int N, bool VS, bool STATS, bool LM, bool GL>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) persistent_kernel(const Plan plan, const Rec<N, VS> *recs, int64_t num,
                                                          uint64_t *counts, uint32_t *status, uint64_t *steps,
                                                          Ctrl *ctrl, Rec<N, VS> *items, uint32_t *ready,
                                                          int64_t item_cap, Tuning tune, const Expand *ex) {
    using S = StackT<N>;
    // LM: line masks in LDS (LdsLane), else in VGPRs (Lane)
    using LaneT = typename std::conditional<LM, LdsLane<N, VS>, VLane<N, VS>>::type;
    constexpr int LINES = LdsLane<N, VS>::LINES;
    if (ex) {
        // the batch as the expansion passes left it
        recs = reinterpret_cast<const Rec<N, VS> *>(ex->recs);
        num = ex->num;
        counts = ex->counts;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    const int nlev = plan.nlev;
    const uint32_t lstride = blockDim.x * 4u;  // LM: bytes between two lines' mask words
    if constexpr (LM) lm_build_desc<N, VS>(plan, smem, lstride);
    else vl_build_desc<N, VS>(plan, smem);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const bool poller = (threadIdx.x >> 6) == 0;  // one wave per workgroup waits for donations
    const uint64_t below = (1ull << lane) - 1ull;
    const uint32_t dbase = lds_of(smem);
    const uint32_t sbase = LM ? lm_stack_base(LINES, nlev, blockDim.x, VS) : kVlStackBase;
    const uint32_t loff = sbase + stack_slot(threadIdx.x, blockDim.x, (uint32_t)sizeof(S));  // from smem
    const uint32_t lane_off = dbase + loff;                             // LDS address
    const uint32_t stride = blockDim.x * (uint32_t)sizeof(S);
    auto slot_of = [&](int l) -> S * { return reinterpret_cast<S *>(smem + (loff + (uint32_t)l * stride)); };
    const int last = nlev - 1;
    const uint64_t cap = (uint64_t)item_cap;
    // donation across the chip is on only with a positive steal_depth
    const int lim = tune.steal_depth > 0 ? nlev - tune.steal_depth : 0;
    const uint64_t total_waves = (uint64_t)gridDim.x * (blockDim.x >> 6);

    // Work moves between the waves of the chip only with global donation;
    // without it, work moves between the waves of a workgroup through the
    // workgroup pool (line masks in VGPRs), and a wave whose lanes are all
    // idle once the static queue is empty leaves when no wave of its
    // workgroup has work left (or at once, without the pool).
    const bool global = GL && cap > 0 && lim > 0;
    // (the pool's addresses are recomputed where used: kept live across the
    // search loop they would cost registers)
    auto rec_area = [&]() { return smem + vl_stacks_end(VLaneDesc<N, VS>::rows(nlev), blockDim.x, sizeof(S)); };
    auto pool_hdr_of = [&]() {
        return reinterpret_cast<uint32_t *>(rec_area() + sizeof(Rec<N, VS>) * blockDim.x / 2);
    };
    auto pool_cap_of = [&]() -> int {
        if (LM || global || tune.wg_pool <= 0) return 0;
        const int room = (int)((sizeof(Rec<N, VS>) * blockDim.x / 2 - kPoolHeader) / sizeof(Rec<N, VS>));
        return tune.wg_pool < room ? tune.wg_pool : room;
    };
    if (pool_cap_of() > 0) {
        // every wave counts as busy until it reaches the tail
        uint32_t *pool_hdr = pool_hdr_of();
        if (threadIdx.x < 2) pool_hdr[threadIdx.x] = 0u;
        if (threadIdx.x < 16) {
            pool_hdr[kPoolIdle + threadIdx.x] = 0u;
            pool_hdr[kPoolBusy + threadIdx.x] = threadIdx.x < (blockDim.x >> 6) ? 64u : 0u;
        }
        __syncthreads();
    }
    // this wave counts as busy from its start until it finds no work anywhere
    if (global && lane == 0) atomicAdd((unsigned long long *)&ctrl->busy, 1ull);
    bool marked = global;

    LaneT L;
    L.cand = 0u;
    L.da = L.da0 = dbase;
    L.sa = lane_off;
    L.cur = {};
    // stack address from descriptor address (see VLane::step, LdsLane::step)
    constexpr uint32_t kDescBytes = LM ? LdsLane<N, VS>::DB : VLane<N, VS>::DB;
    const uint32_t kst = stride / kDescBytes;
    const uint32_t sc0 = lane_off - dbase * kst;
    lds_st<S>(lane_off, (S)0);  // the parked start slot of a lane without a task
    L.cnt = 0;
    L.c32 = 0u;
    if constexpr (LM) L.mbase = dbase + lm_desc_bytes(nlev, VS) + threadIdx.x * 4u;
    const uint32_t da_last = dbase + kDescBytes * (uint32_t)last;
    constexpr bool DSENT = !LM && VLaneDesc<N, VS>::DW;
    bool has = false;           // lane holds a task (possibly finished)
    uint64_t *out = &ctrl->sink;  // where this lane's task count goes (a sink until the first task)
    // start the task of a record / give away part of this lane's task
    // A parked lane's first step reads its start slot (see LdsLane::step).
    // After a task that descended, that slot holds the single bit last taken
    // there; a task that starts without candidates (dead, at the last level,
    // or an empty record) would leave a stale value, so every start clears
    // its slot (a task with candidates overwrites it on its first step).
    auto start = [&](const Rec<N, VS> &r) {
        if constexpr (LM) L.from_rec(r, dbase, last, lane_off, stride, lstride);
        else L.from_rec(r, dbase, last, lane_off, stride);
        lds_st<S>(L.sa, (S)0);
    };
    auto give = [&](int lvl) -> Rec<N, VS> {
        if constexpr (LM) return L.donate(lvl, dbase, slot_of, (uint32_t)(out - counts), lstride);
        else return L.donate(lvl, dbase, slot_of, (uint32_t)(out - counts));
    };
    uint64_t stored = 0;        // part of L.cnt already in *out
    bool static_left = true;    // wave-uniform
    uint64_t cb = 0, ce = 0;    // wave-private range of static tasks
    uint64_t nsteps = 0, nexec = 0;  // DFS steps; steps executed by the lane, parked or not
    uint64_t seen_sig = ~0ull, seen_at = 0;
    uint32_t backoff = 1, tick = 0;
    bool asked = false;         // this (idle poller) wave is counted in ctrl->hungry

    for (;;) {
        // ---------------- search ----------------
        // every lane steps; idle lanes are parked at their start level.
        // Two steps per trip (refill_every rounded up to even) let the
        // register allocator alternate registers instead of copying them.
        if (__ballot(has && !L.done())) {
            for (int it = 0; it < tune.refill_every; it += 2) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    // the steps onto and off the sentinel (D form) are not DFS steps
                    if (STATS) {
                        nsteps += (has && !L.done() && !(DSENT && (L.da == da_last + kDescBytes ||
                                                                  (L.da == da_last && L.cand)))) ? 1u : 0u;
                        ++nexec;
                    }
                    L.template step<S>(kst, sc0, da_last);
                }
            }
        }
        L.flush();
        const bool fin = has && L.done();
        uint64_t want = __ballot(!has || fin);

        if (static_left) {
            // ------------- retire + refill from the static queue -------------
            // While static tasks remain no lane gives work away, so each count
            // has a single writer: a lane whose task finished stores its count
            // (no atomics).  A task still running when the static list runs
            // out has stored nothing; it adds its count atomically when it
            // finishes in the tail (prep zeroed the slot).  Tasks come from a
            // wave-private range refilled with a guided chunk
            // (remaining / (2 * waves), at least chunk_min) by one atomic on
            // ctrl->head.
            if (want && ((int)__popcll(want) >= tune.refill_min || want == ~0ull)) {
                const bool idle = !has || fin;
                const uint64_t k = (uint64_t)__popcll(want);
                const uint64_t rank = (uint64_t)__popcll(want & below);
                const int leader = __ffsll((unsigned long long)want) - 1;
                int64_t my_id = -1;
                uint64_t given = 0;
                while (given < k) {
                    if (cb >= ce) {
                        const uint64_t rem = (uint64_t)num > ce ? (uint64_t)num - ce : 0;
                        uint64_t sz = rem / (2 * total_waves);
                        const uint64_t lo = (uint64_t)tune.chunk_min;
                        sz = sz < lo ? lo : (sz > 65536 ? 65536 : sz);
                        uint64_t base = 0;
                        if (lane == leader)
                            base = atomicAdd((unsigned long long *)&ctrl->head, (unsigned long long)sz);
                        base = bcast64(base, leader);
                        if (base >= (uint64_t)num) {
                            static_left = false;
                            break;
                        }
                        cb = base;
                        ce = base + sz < (uint64_t)num ? base + sz : (uint64_t)num;
                    }
                    const uint64_t take = (k - given) < (ce - cb) ? (k - given) : (ce - cb);
                    if (idle && rank >= given && rank < given + take) my_id = (int64_t)(cb + (rank - given));
                    cb += take;
                    given += take;
                }
                const Rec<N, VS> r = recs[my_id >= 0 ? my_id : 0];
                asm volatile("" ::: "memory");  // keep the load ahead of the store
                if (fin) {
                    *out = L.cnt;
                    has = false;
                }
                if (my_id >= 0) {
                    start(r);
                    out = &counts[r.origin];
                    stored = 0;
                    has = true;
                }
            }
            continue;
        }

        // ================= tail: the static queue is exhausted =================
        // Counts may now have several writers (donated subtrees): add the part
        // not yet stored.
        if (fin) {
            if (L.cnt != stored) atomicAdd((unsigned long long *)out, (unsigned long long)(L.cnt - stored));
            has = false;
            L.cnt = 0;
            stored = 0;
        }
        want = __ballot(!has);
        // ---------------- share work inside the wave ----------------
        // busy lanes hand the untried siblings at their shallowest open level
        // to idle lanes of the same wave, as task records (any number per
        // round)
        int lvl = -1;  // this lane's shallowest open level, or -1
        if (want != ~0ull && (want || pool_cap_of() > 0) && has && !L.done()) {
            const int dep = L.depth(dbase);
            const int top = dep < last - 1 ? dep : last - 1;
            for (int l = L.start_level(dbase); l < top; ++l) {
                const uint32_t sv = *slot_of(l);
                if (sv & (sv - 1u)) {
                    lvl = l;
                    break;
                }
            }
        }
        if (want && want != ~0ull) {
            const uint64_t donors = __ballot(lvl >= 0);
            const uint64_t nd = (uint64_t)__popcll(donors), ni = (uint64_t)__popcll(want);
            uint64_t m = nd < ni ? nd : ni;
            if (!LM) m = m < kMailbox ? m : kMailbox;
            if (m) {
                const uint64_t drank = (uint64_t)__popcll(donors & below);
                const uint64_t rrank = (uint64_t)__popcll(want & below);
                // the idle lane of rank k takes the record of the donor of rank k
                const bool take = !has && rrank < m;
                Rec<N, VS> got;
                if constexpr (LM) {
                    // through registers: LDS sets this layout's occupancy
                    Rec<N, VS> r{};
                    if (lvl >= 0 && drank < m) r = give(lvl);
                    const int src = take ? kth_lane(donors, (uint32_t)rrank) : lane;
                    got = shfl_words(r, src);
                } else {
                    // through the wave's LDS mailbox (cheaper in registers)
                    Rec<N, VS> *mbox = reinterpret_cast<Rec<N, VS> *>(rec_area()) + (threadIdx.x >> 6) * kMailbox;
                    if (lvl >= 0 && drank < m) mbox[drank] = give(lvl);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    if (take) got = mbox[rrank];
                    __builtin_amdgcn_wave_barrier();
                }
                if (take) {
                    start(got);
                    out = &counts[got.origin];
                    stored = 0;
                    has = true;
                }
                if (drank < m) lvl = -1;  // its open level went to a lane of this wave
                want = __ballot(!has);
            }
        }
        if (pool_cap_of() > 0) {
            // ---------------- share work inside the workgroup ----------------
            const int pool_cap = pool_cap_of();
            uint32_t *const pool_hdr = pool_hdr_of();
            Rec<N, VS> *const pool_rec =
                reinterpret_cast<Rec<N, VS> *>(reinterpret_cast<unsigned char *>(pool_hdr) + kPoolHeader);
            const uint32_t my_wave = threadIdx.x >> 6;
            const uint32_t nwaves = blockDim.x >> 6;
            // Each wave publishes its idle and busy lanes.  A wave with idle
            // lanes takes pooled records; a wave whose donors kept their open
            // level (no idle lane of its own left for them) pools it while the
            // other waves have more idle lanes than records are pooled.  The
            // pool is guarded by a lock word; its holder is a wave of this
            // workgroup, resident and never waiting inside the lock.
            const uint32_t nidle = (uint32_t)__popcll(want);
            if (lane == 0) {
                __hip_atomic_store(&pool_hdr[kPoolIdle + my_wave], nidle, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_store(&pool_hdr[kPoolBusy + my_wave], 64u - nidle, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            uint32_t hungry = 0;
            if (lane < (int)nwaves && lane != (int)my_wave)
                hungry = __hip_atomic_load(&pool_hdr[kPoolIdle + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            hungry = (uint32_t)wave_sum64(hungry);
            const uint32_t pcount = (uint32_t)__builtin_amdgcn_readfirstlane(
                (int)__hip_atomic_load(&pool_hdr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            const bool take_round = want && pcount > 0;
            if (!(hungry > pcount && pcount < (uint32_t)pool_cap)) lvl = -1;
            const uint64_t donors = take_round ? 0ull : __ballot(lvl >= 0);
            if (take_round || donors) {
                if (lane == 0) {
                    while (atomicCAS(&pool_hdr[0], 0u, 1u) != 0u) __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)pool_hdr[1]);
                if (take_round) {
                    // the idle lane of rank k takes the k-th of the top m records
                    const uint32_t m = nidle < cnt ? nidle : cnt;
                    const uint32_t rrank = (uint32_t)__popcll(want & below);
                    const bool take = !has && rrank < m;
                    Rec<N, VS> got;
                    if (take) got = pool_rec[cnt - m + rrank];
                    cnt -= m;
                    if (take) {
                        start(got);
                        out = &counts[got.origin];
                        stored = 0;
                        has = true;
                    }
                } else {
                    uint32_t q = hungry > cnt ? hungry - cnt : 0u;
                    const uint32_t room = (uint32_t)pool_cap - cnt;
                    q = q < room ? q : room;
                    const uint32_t drank = (uint32_t)__popcll(donors & below);
                    if (lvl >= 0 && drank < q) pool_rec[cnt + drank] = give(lvl);
                    const uint32_t nd = (uint32_t)__popcll(donors);
                    cnt += nd < q ? nd : q;
                }
                if (lane == 0) pool_hdr[1] = cnt;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) __hip_atomic_store(&pool_hdr[0], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                want = __ballot(!has);
            }
            if (want == ~0ull) {
                // all lanes idle: leave once no other wave of the workgroup has
                // busy lanes and nothing is pooled, else look again shortly
                uint32_t b = 0;
                if (lane < (int)nwaves && lane != (int)my_wave)
                    b = __hip_atomic_load(&pool_hdr[kPoolBusy + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint32_t left = (uint32_t)wave_sum64(b) +
                                      __hip_atomic_load(&pool_hdr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (__builtin_amdgcn_readfirstlane((int)left) == 0) {
                    if (lane == 0)
                        __hip_atomic_store(&pool_hdr[kPoolIdle + my_wave], 0u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            continue;
        }
        if (!global) {
            if (want == ~0ull) break;
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            continue;
        }
        // the queue state is read once every few passes (or when idle)
        ++tick;
        if (want != ~0ull && (tick & (uint32_t)(tune.tail_poll - 1)) != 0) continue;
        uint64_t rsv = 0, hd = 0, busy = 0, hungry = 0;
        if (lane == 0) {
            rsv = ld_relaxed(&ctrl->dq_reserve);
            hd = ld_relaxed(&ctrl->dq_head);
            busy = ld_relaxed(&ctrl->busy);
            hungry = ld_relaxed(&ctrl->hungry);
        }
        rsv = bcast64(rsv, 0);
        hd = bcast64(hd, 0);
        busy = bcast64(busy, 0);
        hungry = bcast64(hungry, 0);
        if (rsv > cap) rsv = cap;
        // ---------------- take donated subtrees ----------------
        if (want && rsv > hd) {
            const uint32_t k = (uint32_t)__popcll(want);
            const int leader = __ffsll((unsigned long long)want) - 1;
            uint64_t h0 = 0, got = 0;
            if (lane == leader) {
                uint64_t h = hd;
                for (int tries = 0; tries < 16; ++tries) {
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
                if (got && !marked) atomicAdd((unsigned long long *)&ctrl->busy, 1ull);
                if (got && asked) atomicAdd((unsigned long long *)&ctrl->hungry, ~0ull);  // -1
            }
            h0 = bcast64(h0, leader);
            got = bcast64(got, leader);
            if (got) {
                marked = true;
                asked = false;
                backoff = 1;
            }
            if (!has) {
                const uint64_t rank = (uint64_t)__popcll(want & below);
                if (rank < got) {
                    const uint64_t slot = h0 + rank;
                    // the slot's writer publishes it right after reserving it
                    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                    bool ok = false;
                    for (;;) {
                        if (__hip_atomic_load(&ready[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) {
                            ok = true;
                            break;
                        }
                        if (__builtin_amdgcn_s_memrealtime() - t0 > kStallTicks) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    if (ok) {
                        __threadfence();
                        const Rec<N, VS> r = items[slot];
                        __hip_atomic_store(&ready[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        start(r);
                        out = &counts[r.origin];
                        stored = 0;
                        has = true;
                    } else if (status) {
                        atomicOr(status, 2u);
                    }
                }
            }
            want = __ballot(!has);
        }
        // ---------------- termination ----------------
        if (want == ~0ull) {
            if (marked) {
                __threadfence();
                if (lane == 0) atomicAdd((unsigned long long *)&ctrl->busy, ~0ull);  // -1
                marked = false;
            }
            // a wave that is not its workgroup's poller leaves as soon as it
            // is idle: the busy waves and the pollers finish the tail
            if (!poller || (busy == 0 && hd >= rsv)) {
                if (asked && lane == 0) atomicAdd((unsigned long long *)&ctrl->hungry, ~0ull);
                break;
            }
            if (!asked) {
                if (lane == 0) atomicAdd((unsigned long long *)&ctrl->hungry, 1ull);
                asked = true;
            }
            const uint64_t sig = busy ^ (rsv << 20) ^ (hd << 40);
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (sig != seen_sig) {
                seen_sig = sig;
                seen_at = now;
            } else if (now - seen_at > kStallTicks) {
                if (lane == 0 && status) atomicOr(status, 2u);
                break;
            }
            for (uint32_t t = 0; t < backoff; ++t) __builtin_amdgcn_s_sleep(64);
            backoff = backoff < 32 ? backoff * 2 : 32;
            continue;
        }
        // ---------------- donate to idle waves elsewhere ----------------
        // only full waves give work away across the chip, only large subtrees
        // (levels above the cut-off), and only as many as idle pollers ask for
        if (cap > 0 && lim > 0 && want == 0 && hungry > rsv - hd) {
            int lvl = -1;
            if (!L.done()) {
                const int dep = L.depth(dbase);
                const int top = dep < lim ? dep : lim;
                for (int l = L.start_level(dbase); l < top; ++l) {
                    const uint32_t sv = *slot_of(l);
                    if (sv & (sv - 1u)) {
                        lvl = l;
                        break;
                    }
                }
            }
            const uint64_t donors = __ballot(lvl >= 0);
            uint64_t quota = hungry - (rsv - hd);
            quota = quota < (uint64_t)tune.donate_max ? quota : (uint64_t)tune.donate_max;
            if (lvl >= 0 && (uint64_t)__popcll(donors & below) < quota) {
                const uint64_t slot = atomicAdd((unsigned long long *)&ctrl->dq_reserve, 1ull);
                if (slot < cap) {
                    items[slot] = give(lvl);
                    __threadfence();
                    __hip_atomic_store(&ready[slot], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        // the tail is rare: let every memory access of this pass finish here so
        // that the search loop never waits on one
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
    }
    if (STATS && steps) {
        atomicAdd((unsigned long long *)steps, (unsigned long long)nsteps);
        atomicAdd((unsigned long long *)(steps + 1), (unsigned long long)nexec);
    }
}

// ---------------------------------------------------------------------------
// breadth-first expansion of small batches
// ---------------------------------------------------------------------------
// A batch with fewer tasks than lanes leaves most of the GPU idle.  Before the
// persistent kernel runs, passes replace every task by its children one level
// deeper (the split of Sec. 5.2, done on the device), until the batch has
// `target` tasks or the next level would not fit the buffers.  Children on
// the last level are counted at once; dead children are dropped.
//
// A pass is two kernels over kExBlocks workgroups, each taking an equal
// contiguous share of the current tasks: ex_tally stores the number of live
// children of each share, ex_write derives every share's output offset from
// those tallies and writes the children in order.  No atomics or fences
// place the output, so tasks stay sorted by prefix.  The pass state is double
// buffered (pass p reads state p & 1 and workgroup 0 writes state (p+1) & 1),
// so every decision is taken on the device and the sequence needs no host
// round trip: it can be captured in a graph.
//
// Expanded tasks have their own count slots (tcounts), zeroed when the task
// is written (the search adds to a slot atomically when it takes a task at
// the end of the static queue) and summed into the prefixes' counts by
// ex_scatter at the end.

__global__ void ex_init(Expand *E, const void *recs, int64_t num, uint64_t *counts) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Expand e;
        e.recs = recs;
        e.num = num;
        e.counts = counts;
        e.orig = nullptr;
        e.want = e.want_next = e.nout = 0;
        e.cur = 0;
        e.stop = num == 0;
        e.done = e.pad = 0;
        E[0] = e;
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += (uint32_t)__shfl_xor((int)x, o);
    return x;
}

// 64-bit value of lane (this lane's DPP source) added to x; lanes outside
// row_mask add 0
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_add64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK, 0xF, false);
    return x + (((uint64_t)hi << 32) | lo);
}

// Sum over the wave by DPP lane moves: swaps within pairs and quads, the
// half-row and row mirrors (every lane of a 16-lane row then holds the row's
// sum), then the row broadcasts of lanes 15 and 31 into the rows above.  The
// total ends in lane 63.  Every lane of the wave must be active.
__device__ __forceinline__ uint64_t wave_sum64_last(uint64_t x) {
    x = dpp_add64<0xB1>(x);         // quad_perm [1,0,3,2]
    x = dpp_add64<0x4E>(x);         // quad_perm [2,3,0,1]
    x = dpp_add64<0x141>(x);        // row_half_mirror
    x = dpp_add64<0x140>(x);        // row_mirror
    x = dpp_add64<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x = dpp_add64<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// the same total in every lane
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) { return bcast64(wave_sum64_last(x), 63); }

// Inclusive sum over the workgroup (W waves of 64 lanes); *total gets the
// workgroup's sum.  Uses part[W] of LDS; every thread must call it.
template <int W = 4>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *part, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) part[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const uint32_t q = part[k];
        before += k < w ? q : 0u;
        all += q;
    }
    __syncthreads();  // part[] may be reused right after
    *total = all;
    return x + before;
}

// Adds values to ucounts[orig] for (orig, value) pairs that a wave visits in
// increasing position order.  Tasks are sorted by prefix, so the values of
// one prefix are summed in registers and added with one atomic per run.  The
// run state is wave-uniform.
struct RunSum {
    uint32_t o = 0xFFFFFFFFu;
    uint64_t v = 0;

    __device__ __forceinline__ void add(uint32_t orig, uint64_t val, uint64_t *ucounts) {
        const int lane = threadIdx.x & 63;
        uint64_t pend = __ballot(val != 0);
        while (pend) {
            const int ld = __ffsll((unsigned long long)pend) - 1;
            const uint32_t g = (uint32_t)__shfl((int)orig, ld);
            const bool in = ((pend >> lane) & 1ull) && orig == g;
            const uint64_t grp = __ballot(in);
            const uint64_t sum = wave_sum64(in ? val : 0ull);
            if (g != o) {
                if (lane == 0 && v) atomicAdd((unsigned long long *)&ucounts[o], (unsigned long long)v);
                o = g;
                v = 0;
            }
            v += sum;
            pend &= ~grp;
        }
    }

    // one atomic per run left in the workgroup's W waves (runs of equal
    // prefixes merged); every thread must call it
    template <int W = 4>
    __device__ __forceinline__ void flush(uint64_t *ucounts, uint32_t *so, uint64_t *sv) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (lane == 0) {
            so[w] = o;
            sv[w] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t co = 0xFFFFFFFFu;
            uint64_t cv = 0;
            for (int k = 0; k < W; ++k) {
                if (!sv[k]) continue;
                if (so[k] != co) {
                    if (cv) atomicAdd((unsigned long long *)&ucounts[co], (unsigned long long)cv);
                    co = so[k];
                    cv = 0;
                }
                cv += sv[k];
            }
            if (cv) atomicAdd((unsigned long long *)&ucounts[co], (unsigned long long)cv);
        }
        v = 0;
    }
};

// Children of one task: how many are live (to be written) and, when they sit
// on the last level, their candidate counts (squares completed at once).
template <int N, bool VS>
struct Kids {
    Lane<N, VS> L;
    uint32_t cand = 0u, lvl = kNone, kids = 0u, orig = 0u;
    uint64_t leaves = 0u;

    __device__ __forceinline__ void load(const Rec<N, VS> *in, const uint32_t *iorig, int64_t i,
                                         const uint32_t *sdesc, int last) {
        const Rec<N, VS> r = in[i];
        lvl = r.cl >> 16;
        if (lvl == kNone) return;
        orig = iorig ? iorig[i] : (uint32_t)i;
        if ((int)lvl >= last) {  // not produced by prep or by a pass; counted as the search would
            leaves = (uint64_t)__builtin_popcount(r.cl & 0xFFFFu);
            lvl = kNone;
            return;
        }
        L.from_rec(r, sdesc, last);
        cand = r.cl & 0xFFFFu;
        const uint32_t dc = sdesc[lvl], dn = sdesc[lvl + 1];
        for (uint32_t c = cand; c; c &= c - 1u) {
            Lane<N, VS> T = L;
            T.toggle(dc, c & (0u - c));
            const uint32_t nc = T.cands(dn);
            if ((int)lvl + 1 == last) leaves += (uint64_t)__builtin_popcount(nc);
            else kids += nc ? 1u : 0u;
        }
    }
};

__device__ __forceinline__ void ex_share(int64_t num, int64_t *b0, int64_t *b1) {
    const int64_t per = (num + kExBlocks - 1) / kExBlocks;
    const int64_t lo = (int64_t)blockIdx.x * per;
    *b0 = lo < num ? lo : num;
    *b1 = lo + per < num ? lo + per : num;
}

template <int N, bool VS>
__global__ void __launch_bounds__(256) ex_tally(const Plan plan, const Expand *E2, int pass, uint32_t *blk) {
    __shared__ uint32_t sdesc[kMaxLevels];
    __shared__ uint32_t part[4];
    const Expand *E = &E2[pass & 1];
    if (E->stop) return;
    const int nlev = plan.nlev;
    for (int k = threadIdx.x; k < nlev; k += blockDim.x) sdesc[k] = plan.desc[k];
    __syncthreads();
    const Rec<N, VS> *in = reinterpret_cast<const Rec<N, VS> *>(E->recs);
    const uint32_t *iorig = E->orig;
    int64_t b0, b1;
    ex_share(E->num, &b0, &b1);
    uint32_t mine = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        Kids<N, VS> k;
        k.load(in, iorig, i, sdesc, nlev - 1);
        mine += k.kids;
    }
    uint32_t total = 0;
    block_scan(mine, part, &total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

template <int N, bool VS>
__global__ void __launch_bounds__(256) ex_write(const Plan plan, Expand *E2, int pass, const uint32_t *blk,
                                                void *buf1, void *buf2, uint32_t *orig1, uint32_t *orig2,
                                                uint64_t *ucounts, uint64_t *tcounts, uint32_t *status,
                                                int64_t target, int64_t cap) {
    using R = Rec<N, VS>;
    static_assert(kExBlocks == 4 * 256, "each thread sums four tallies");
    __shared__ uint32_t sdesc[kMaxLevels];
    __shared__ uint32_t part[4];
    __shared__ uint32_t so[4];
    __shared__ uint64_t sv[4];
    const Expand e = E2[pass & 1];
    Expand *eo = &E2[(pass + 1) & 1];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (e.stop) {
        if (lead) *eo = e;
        return;
    }
    const int nlev = plan.nlev;
    for (int k = threadIdx.x; k < nlev; k += blockDim.x) sdesc[k] = plan.desc[k];
    // output offset of this share and the pass total, from the tallies
    uint32_t t_all = 0, t_before = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t h = 4u * threadIdx.x + (uint32_t)k;
        const uint32_t q = blk[h];
        t_all += q;
        t_before += h < blockIdx.x ? q : 0u;
    }
    uint32_t total = 0, base = 0;
    block_scan(t_all, part, &total);
    block_scan(t_before, part, &base);
    const int cur = e.cur;
    R *out = reinterpret_cast<R *>(cur == 1 ? buf2 : buf1);
    uint32_t *oorig = cur == 1 ? orig2 : orig1;
    const bool go = e.num < target && (int64_t)total <= cap;
    if (lead) {
        Expand n = e;
        if (go) {
            n.recs = out;
            n.orig = oorig;
            n.cur = cur == 1 ? 2 : 1;
            n.num = total;
            n.counts = tcounts;
            n.stop = total == 0;
        } else {
            n.stop = 1;
        }
        *eo = n;
    }
    if (!go) return;
    const R *in = reinterpret_cast<const R *>(e.recs);
    const int last = nlev - 1;
    int64_t b0, b1;
    ex_share(e.num, &b0, &b1);
    uint64_t run = base;
    RunSum acc;
    for (int64_t chunk = b0; chunk < b1; chunk += blockDim.x) {  // uniform per workgroup
        const int64_t i = chunk + threadIdx.x;
        Kids<N, VS> k;
        if (i < b1) k.load(in, e.orig, i, sdesc, last);
        uint32_t step = 0;
        const uint32_t incl = block_scan(k.kids, part, &step);
        uint64_t pos = run + (incl - k.kids);
        run += step;
        if (k.kids) {
            const uint32_t dc = sdesc[k.lvl], dn = sdesc[k.lvl + 1];
            for (uint32_t c = k.cand; c; c &= c - 1u) {
                Lane<N, VS> T = k.L;
                T.toggle(dc, c & (0u - c));
                const uint32_t nc = T.cands(dn);
                if (!nc) continue;
                if (pos >= (uint64_t)cap) {  // cannot happen: the tallies bound the output
                    if (status) atomicOr(status, 4u);
                    break;
                }
                R o;
#pragma unroll
                for (int w = 0; w < Geo<N, VS>::WR; ++w) o.R[w] = T.R[w];
#pragma unroll
                for (int w = 0; w < Geo<N, VS>::WC; ++w) o.C[w] = T.C[w];
                o.diag = T.md | (T.ad << 16);
                o.cl = nc | ((k.lvl + 1u) << 16);
                o.origin = (uint32_t)pos;
                o.pad = 0;
                out[pos] = o;
                oorig[pos] = k.orig;
                // the search may add to a task's slot before it stores one
                tcounts[pos] = 0;
                ++pos;
            }
        }
        acc.add(k.orig, k.leaves, ucounts);
    }
    acc.flush(ucounts, so, sv);
}

// The narrow first levels of a small batch, all inside one workgroup of
// 1024 lanes: each level is processed in chunks of 1024 tasks with a
// workgroup scan placing the children, so a level costs a few microseconds
// instead of two kernel launches.  Runs from state 0 until the batch has
// `limit` tasks (the multi-workgroup passes take over from there), reaches
// the target, or has no live task left, and leaves the result in state 0.
// The host keeps N * limit <= cap, so a level always fits the buffers.
template <int N, bool VS>
__global__ void __launch_bounds__(1024) ex_small(const Plan plan, Expand *E2, void *buf1, void *buf2,
                                                 uint32_t *orig1, uint32_t *orig2, uint64_t *ucounts,
                                                 uint64_t *tcounts, uint32_t *status, int64_t target, int64_t cap,
                                                 int64_t limit, int max_passes) {
    using R = Rec<N, VS>;
    constexpr int W = 16;
    __shared__ uint32_t sdesc[kMaxLevels];
    __shared__ uint32_t part[W];
    __shared__ uint32_t so[W];
    __shared__ uint64_t sv[W];
    const int nlev = plan.nlev;
    for (int k = threadIdx.x; k < nlev; k += blockDim.x) sdesc[k] = plan.desc[k];
    __syncthreads();
    const int last = nlev - 1;
    Expand e = E2[0];
    RunSum acc;
    for (int p = 0; p < max_passes && !e.stop && e.num < target && e.num < limit; ++p) {
        const int cur = e.cur;
        R *out = reinterpret_cast<R *>(cur == 1 ? buf2 : buf1);
        uint32_t *oorig = cur == 1 ? orig2 : orig1;
        const R *in = reinterpret_cast<const R *>(e.recs);
        uint64_t run = 0;
        for (int64_t chunk = 0; chunk < e.num; chunk += blockDim.x) {  // uniform
            const int64_t i = chunk + threadIdx.x;
            Kids<N, VS> k;
            if (i < e.num) k.load(in, e.orig, i, sdesc, last);
            uint32_t step = 0;
            const uint32_t incl = block_scan<W>(k.kids, part, &step);
            uint64_t pos = run + (incl - k.kids);
            run += step;
            if (k.kids) {
                const uint32_t dc = sdesc[k.lvl], dn = sdesc[k.lvl + 1];
                for (uint32_t c = k.cand; c; c &= c - 1u) {
                    Lane<N, VS> T = k.L;
                    T.toggle(dc, c & (0u - c));
                    const uint32_t nc = T.cands(dn);
                    if (!nc) continue;
                    if (pos >= (uint64_t)cap) {  // cannot happen: N * limit <= cap
                        if (status) atomicOr(status, 4u);
                        break;
                    }
                    R o;
#pragma unroll
                    for (int w = 0; w < Geo<N, VS>::WR; ++w) o.R[w] = T.R[w];
#pragma unroll
                    for (int w = 0; w < Geo<N, VS>::WC; ++w) o.C[w] = T.C[w];
                    o.diag = T.md | (T.ad << 16);
                    o.cl = nc | ((k.lvl + 1u) << 16);
                    o.origin = (uint32_t)pos;
                    o.pad = 0;
                    out[pos] = o;
                    oorig[pos] = k.orig;
                    tcounts[pos] = 0;
                    ++pos;
                }
            }
            acc.add(k.orig, k.leaves, ucounts);
        }
        __syncthreads();  // this level's children are written before they are read
        e.recs = out;
        e.orig = oorig;
        e.cur = cur == 1 ? 2 : 1;
        e.num = (int64_t)run;
        e.counts = tcounts;
        e.stop = run == 0;
    }
    acc.flush<W>(ucounts, so, sv);
    if (threadIdx.x == 0) E2[0] = e;
}

// add the expanded tasks' counts to their prefixes
__global__ void __launch_bounds__(256) ex_scatter(const Expand *E, uint64_t *ucounts) {
    __shared__ uint32_t so[4];
    __shared__ uint64_t sv[4];
    const uint32_t *orig = E->orig;
    if (!orig) return;  // nothing was expanded: the search wrote ucounts itself
    const uint64_t *tc = E->counts;
    int64_t b0, b1;
    ex_share(E->num, &b0, &b1);
    RunSum acc;
    for (int64_t chunk = b0; chunk < b1; chunk += blockDim.x) {
        const int64_t i = chunk + threadIdx.x;
        const bool ok = i < b1;
        acc.add(ok ? orig[i] : 0u, ok ? tc[i] : 0ull, ucounts);
    }
    acc.flush(ucounts, so, sv);
}

// ready flags of the slots the previous launch on this queue reserved (all
// consumed after a normal end; cleared anyway in case that launch stopped
// early)
__global__ void reset_queue(const Ctrl *ctrl, uint32_t *ready, int64_t cap) {
    const uint64_t r = ctrl->dq_reserve;
    const int64_t used = (int64_t)(r < (uint64_t)cap ? r : (uint64_t)cap);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t k = t; k < used; k += (int64_t)gridDim.x * blockDim.x) ready[k] = 0u;
}

__global__ void init_ctrl(Ctrl *ctrl) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->head = 0;
        ctrl->dq_reserve = 0;
        ctrl->dq_head = 0;
        ctrl->busy = 0;
        ctrl->sink = 0;
        ctrl->hungry = 0;
    }
}

__global__ void zero_u64(uint64_t *p, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t k = t; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = 0;
}

// out = sum_k mult[k] * counts[k] (mult == nullptr: all 1).  A first kernel
// zeroes out; the second runs one workgroup of 1024 per CU over the array
// (grid-stride, four counts per thread and step): each wave sums by DPP lane
// moves, the workgroup's waves through LDS, and one atomic per workgroup adds
// the result (atomics on one address are serialised, so their number is kept
// to the number of CUs).  Only kernels: the pair can be captured in a graph.
__global__ void zero_one(uint64_t *out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = 0;
}

constexpr int kReduceBlock = 1024;

__global__ void __launch_bounds__(kReduceBlock) reduce_weighted(const uint64_t *__restrict__ counts,
                                                                const uint32_t *__restrict__ mult, int64_t num,
                                                                uint64_t *out) {
    __shared__ uint64_t part[kReduceBlock / 64];
    // two 16-byte count loads and one 16-byte weight load per step when both
    // arrays are 16-byte aligned
    const bool vec = ((uintptr_t)counts % 16 == 0) && ((uintptr_t)mult % 16 == 0);
    const int64_t nv = vec ? num / 4 : 0;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    for (int64_t q = t0; q < nv; q += nt) {
        const ulonglong2 c0 = reinterpret_cast<const ulonglong2 *>(counts)[2 * q];
        const ulonglong2 c1 = reinterpret_cast<const ulonglong2 *>(counts)[2 * q + 1];
        if (mult) {
            const uint4 m = reinterpret_cast<const uint4 *>(mult)[q];
            acc += c0.x * m.x + c0.y * m.y + c1.x * m.z + c1.y * m.w;
        } else {
            acc += c0.x + c0.y + c1.x + c1.y;
        }
    }
    for (int64_t k = 4 * nv + t0; k < num; k += nt) acc += counts[k] * (mult ? (uint64_t)mult[k] : 1ull);
    acc = wave_sum64_last(acc);
    if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x < 64) {
        uint64_t v = threadIdx.x < blockDim.x / 64 ? part[threadIdx.x] : 0ull;
        v = wave_sum64_last(v);
        if (threadIdx.x == 63 && v) atomicAdd((unsigned long long *)out, (unsigned long long)v);
    }
}

// integer VALU probe: 8 independent dependency chains of 32-bit xor/add/shift per lane
__global__ void __launch_bounds__(256) valu_probe(int iters, uint32_t *sink) {
    uint32_t a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = threadIdx.x * 2654435761u + k;
    const uint32_t m = blockIdx.x | 1u;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = (a[k] ^ m) + 0x9E3779B9u;
            a[k] = (a[k] << 1) + (a[k] >> 31);
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r ^= a[k];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// ---------------------------------------------------------------------------
// serving kernel: continuous batching of counting jobs on the device
// ---------------------------------------------------------------------------
// One long-running grid (one launch serves many jobs of any order 4..9 and
// flags) built from the persistent lane machinery above.  The host publishes
// jobs into a ring of slots in host-pinned memory; a job is one request's
// prefix split into workunits (Sec. 5.2), whose cells sit in a host-pinned
// prefix pool.  Every wave works on one job at a time: it copies the job's
// fill order into its own descriptor table in LDS, takes chunks of the job's
// workunits (a compare-and-swap on the job's head, which carries the job
// number, so a slot reused for a later job is never taken from by mistake),
// turns each into a task record in registers as it starts it, refills idle
// lanes and, once the job has no untaken workunit, shares subtrees inside the
// wave.  A finished piece adds its count to the job's total and takes one off
// the job's outstanding counter; the piece that takes it to zero writes the
// job's result to host-pinned memory.  A wave whose job has nothing left to
// take moves, when all its lanes are idle, to the oldest published job that
// has.  Waves of different jobs -- and of different orders -- run side by
// side, so jobs that arrive while others run are taken as soon as waves free
// up.
//
// The grid leaves as a whole, never wave by wave: a gate word counts the
// waves inside a job, and a wave that has found no job for idle_ticks closes
// the gate only while that count is zero (one compare-and-swap from 0 to the
// closing bit); a wave enters a job by adding one and goes on only if the
// closing bit was clear.  Once closed, every wave leaves at its next look,
// and the host launches the grid again for the next job.  (Were
// waves to leave one by one, a grid that had thinned out during a long job's
// tail would keep serving every later job with the few waves left, and the
// host, seeing the kernel still running, would not launch it again.)  The
// stop flag ends every wave that is not inside a job.
//
// LDS per wave: its descriptor table, the first level's 4-byte descriptor and
// pattern of the job (for building records), its lanes' stacks (one row of
// 64 slots per level), a 32-record mailbox for sharing subtrees (a pass
// shares at most 32: donors are busy lanes, takers idle ones) and, for
// order 9 without vertical symmetry, its lanes' line masks (the LDS-mask
// layout: one 4-byte word per line and lane, lines 256 bytes apart).
constexpr uint32_t kSvTable = 16u * 65u;  // >= 16 B x (64 + 1) (even N <= 8), 8 B x (81 + 1) (N = 9)
constexpr uint32_t kSvInfo = 64u;         // patbits[8], first descriptor, levels
constexpr uint32_t kSvStacks = 82u * 128u;  // (81 + 1) rows x 64 lanes x 2 bytes
constexpr uint32_t kSvMbox = 32u * 48u;     // 32 records of order 9
constexpr uint32_t kSvLine = 64u * 4u;      // bytes between two lines' mask words
constexpr uint32_t kSvMasks = 9u * kSvLine; // 9 packed lines (order 9)
constexpr uint32_t kSvWave = kSvTable + kSvInfo + kSvStacks + kSvMbox + kSvMasks;
constexpr int kSvBlock = 256;
constexpr uint32_t kSvPoll = 4;   // passes between a full wave's looks at the donation queue
constexpr int kSvShareMin = 8;    // idle lanes that start sharing inside a wave
// Subtrees a wave hands on per look: one.  A lane that reserves record q
// waits until record q - kServeItems of the same entry is read; were two
// lanes of one wave to reserve q - kServeItems and q in the same pass, the
// second would wait for a record its own wave has not yet written.
constexpr int kSvDonate = 1;
static_assert(kSvWave % 16 == 0, "per-wave LDS regions keep 16-byte alignment");

// system-scope loads of the host-pinned ring (no cached copy is ever used)
__device__ __forceinline__ uint32_t hload32(const void *p) {
    return __hip_atomic_load(reinterpret_cast<const uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t hload64(const void *p) {
    return __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Works the job of ring slot `slot` whose pub word is `pub` with this wave
// until the job has no untaken workunit and every lane of the wave is idle.
// Returns whether the wave took any workunit.
template <int N, bool VS>
__device__ __noinline__ bool serve_job(const ServeArgs &a, int slot, uint64_t pub, unsigned char *wsm, int lane) {
    using S = StackT<N>;
    using DT = VLaneDesc<N, VS>;
    using R = Rec<N, VS>;
    using G = Geo<N, VS>;
    // order 9 (plain; with vertical symmetry every order-9 count is 0 and is
    // answered on the host) keeps its line masks in LDS, as the batch path
    // does from order 9 on; smaller orders keep them in VGPRs
    constexpr bool LM = N >= 9 && !VS;
    using LaneT = typename std::conditional<LM, LdsLane<N, VS>, VLane<N, VS>>::type;
    static_assert(!LM || LdsLane<N, VS>::LINES * kSvLine <= kSvMasks, "line masks");
    constexpr uint32_t DB = LM ? LdsLane<N, VS>::DB : DT::DB;
    constexpr int NN = N * N;
    constexpr int PS = (NN + 15) & ~15;  // pre_stride(N)
    static_assert(DB * (uint32_t)(NN + 1) <= kSvTable, "descriptor table");
    static_assert((uint32_t)(NN + 1) * 64u * sizeof(S) <= kSvStacks, "stacks");
    static_assert(32u * sizeof(R) <= kSvMbox, "mailbox");
    static_assert(sizeof(R) <= (size_t)kServeItemBytes, "donation record");
    const uint64_t below = (1ull << lane) - 1ull;
    const JobDesc *jd = &a.jobs[slot];
    JobState *js = &a.state[slot];
    const uint64_t seq32 = pub >> 32;                 // job number
    const int64_t ntasks = (int64_t)(pub & 0xFFFFFFFFull);  // its workunits
    const int nlev = (int)hload32(&jd->plan.nlev);
    if (nlev < 0 || nlev > NN) return false;  // never for a published job; keeps the table in bounds
    // launch parameters in uniform registers (not re-read from the argument
    // struct inside the search loop)
    const int refill_every = __builtin_amdgcn_readfirstlane(a.refill_every);
    const uint64_t chunk = (uint64_t)__builtin_amdgcn_readfirstlane(a.chunk);
    JobDone *done_rec = &a.done[slot];
    const int last = nlev - 1;
    const uint8_t *pre = a.pool + (int64_t)hload64(&jd->pre_off);
    // the job's donation queue, a ring of kServeItems records: record q
    // lives in entry q % kServeItems; the entry's ready word holds
    // job number << 32 | (2 x lap + 1) once record q (lap q / kServeItems)
    // is written and 2 x lap + 2 once it is read, so an entry is refilled
    // only after its previous record of the same job was read
    R *items = reinterpret_cast<R *>(a.items + (size_t)slot * ((size_t)kServeItems * kServeItemBytes));
    uint64_t *ready = a.ready + (size_t)slot * kServeItems;
    const uint64_t tag = seq32 << 32;
    // donated subtrees start above this level (off unless steal_depth > 0)
    const int lim = a.steal_depth > 0 ? nlev - a.steal_depth : 0;
    uint32_t tick = 0;

    // the job's plan into this wave's LDS: descriptor table, pattern, first level
    const uint32_t dbase = lds_of(wsm);
    uint32_t *info = reinterpret_cast<uint32_t *>(wsm + kSvTable);
    for (int k = lane; k < nlev; k += 64) {
        const uint32_t d = hload32(&jd->plan.desc[k]);
        const uint32_t keep = (N <= 8 && k != nlev - 1) ? G::ALL : 0u;
        if constexpr (LM) {
            // row and column word offsets of the level's cell, then its diagonals
            const uint32_t i = ((d >> 6) & 3u) * G::LPW + (d & 63u) / N;
            const uint32_t j = ((d >> 14) & 3u) * G::LPW + ((d >> 8) & 63u) / N;
            const uint32_t roff = i * kSvLine, coff = (LdsLane<N, VS>::PACK ? j : N + j) * kSvLine;
            reinterpret_cast<uint2 *>(wsm)[k] =
                make_uint2(roff | (coff << 16), (d_md(d) & G::ALL) | ((d_ad(d) & G::ALL) << 16));
        } else if constexpr (DT::DW) {
            const uint32_t z = (d >> 16) & 1u ? 0u : ((d >> 17) & 1u ? 8u : kDwNone);
            reinterpret_cast<uint4 *>(wsm)[k] = make_uint4(d & 63u, (d >> 8) & 63u, z, 0u);
        } else {
            reinterpret_cast<uint2 *>(wsm)[k] = make_uint2((d & 0xFFu) | ((d_md(d) & G::ALL) << 16),
                                                           ((d >> 8) & 0xFFu) | (keep << 8) | ((d_ad(d) & G::ALL) << 16));
        }
    }
    if constexpr (DT::DW) {
        if (lane == 0) reinterpret_cast<uint4 *>(wsm)[nlev] = make_uint4(0u, 0u, kDwSentinel, 1u);
    }
    if (lane < 8) info[lane] = hload32(&jd->plan.patbits[lane]);
    if (lane == 8) info[8] = nlev > 0 ? hload32(&jd->plan.desc[0]) : 0u;
    const uint32_t loff = kSvTable + kSvInfo + (uint32_t)lane * (uint32_t)sizeof(S);
    const uint32_t lane_off = dbase + loff;
    const uint32_t stride = 64u * (uint32_t)sizeof(S);
    const uint32_t kst = stride / DB;
    const uint32_t sc0 = lane_off - dbase * kst;
    auto slot_of = [&](int l) -> S * { return reinterpret_cast<S *>(wsm + (loff + (uint32_t)l * stride)); };
    // the shallowest level in [from, top) whose stack entry still holds
    // more than one candidate, or -1: eight independent LDS reads at a time
    auto open_level = [&](int from, int top) -> int {
        for (int l0 = from; l0 < top; l0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = l0 + u < top ? (uint32_t)*slot_of(l0 + u) : 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (v[u] & (v[u] - 1u)) return l0 + u;
        }
        return -1;
    };
    R *mbox = reinterpret_cast<R *>(wsm + kSvTable + kSvInfo + kSvStacks);
    const uint32_t da_last = dbase + DB * (uint32_t)(last > 0 ? last : 0);
    lds_st<S>(lane_off, (S)0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    uint32_t patbits[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) patbits[k] = info[k];
    const uint32_t desc0 = info[8];

    LaneT L;
    if constexpr (LM) {
        L.md = L.ad2 = 0u;
        L.mbase = dbase + kSvTable + kSvInfo + kSvStacks + kSvMbox + (uint32_t)lane * 4u;
        L.cur = lds_ld2(dbase);
    } else {
#pragma unroll
        for (int k = 0; k < G::WR; ++k) L.R[k] = 0;
#pragma unroll
        for (int k = 0; k < G::WC; ++k) L.C[k] = 0;
        L.mdh = L.adh = 0u;
        L.cur = DT::load(dbase);
    }
    L.cand = 0u;
    L.da = L.da0 = dbase;
    L.sa = lane_off;
    L.cnt = 0;
    L.c32 = 0u;
    bool has = false;
    bool job_left = true;
    bool took = false;
    // Pieces of the job this wave holds (workunits and records it took) and
    // each lane's squares over them: released together once every lane is
    // idle.  Subtrees shared among the wave's own lanes stay inside those
    // pieces and cost no atomic.
    uint64_t own = 0;
    uint64_t acc = 0;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / 64u);
    uint64_t share = (uint64_t)ntasks / (2u * nwaves);
    share = share < chunk ? share : chunk;
    share = share > 1u ? share : 1u;
    auto start = [&](const R &r) {
        if constexpr (LM) L.from_rec(r, dbase, last, lane_off, stride, kSvLine);
        else L.from_rec(r, dbase, last, lane_off, stride);
        lds_st<S>(L.sa, (S)0);
    };
    auto give = [&](int lvl) -> R {
        if constexpr (LM) return L.donate(lvl, dbase, slot_of, 0u, kSvLine);
        else return L.donate(lvl, dbase, slot_of, 0u);
    };

    for (;;) {
        if (__ballot(has && !L.done())) {
            for (int it = 0; it < refill_every; it += 2) {
#pragma unroll
                for (int u = 0; u < 2; ++u) L.template step<S>(kst, sc0, da_last);
            }
        }
        L.flush();
        if (has && L.done()) {
            acc += L.cnt;
            L.cnt = 0;
            has = false;
        }
        uint64_t want = __ballot(!has);
        if (want == ~0ull && own) {
            // Every lane is idle: all the work of the pieces this wave took is
            // done.  Their count goes into the job's total, then `own` pieces
            // less are outstanding.  Both are device-scope atomics performed
            // where every wave's atomics meet; the decrement's operand depends
            // on the add's result, so the add is done before the decrement is
            // issued, and the wave that takes the counter to zero finds every
            // piece's count in the total (no cache write-back or invalidation
            // on this path).
            const uint64_t sum = wave_sum64(acc);
            acc = 0;
            if (lane == 0) {
                const uint64_t prev =
                    __hip_atomic_fetch_add(&js->total, sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // -own, computed from the add's result (a total never reaches 2^64 - 1)
                const uint64_t dec = prev == ~0ull ? 0ull : 0ull - own;
                const uint64_t left =
                    __hip_atomic_fetch_add(&js->remaining, dec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (left == own) {
                    // the job's last pieces: its result to host-pinned memory
                    JobDone *d = done_rec;
                    const uint64_t tot =
                        __hip_atomic_fetch_add(&js->total, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t ts = __hip_atomic_load(&js->t_start, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t nr =
                        __hip_atomic_load(&js->dq_res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 0xFFFFFFFFull;
                    __hip_atomic_store(&d->shared, nr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(&d->total, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(&d->t_start, ts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(&d->t_end, (uint64_t)__builtin_amdgcn_s_memrealtime(), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(&d->pub, pub, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
            own = 0;
        }

        // ---------------- a full wave gives subtrees to waves without work ----------------
        // Every kSvPoll passes a wave with fewer than kSvShareMin idle lanes
        // (it shares inside itself from that many on) compares the
        // number of waves that found no work with the records waiting in the
        // job's queue; for the difference (at most kSvDonate per wave and
        // look) its lanes hand on the untried siblings at their shallowest
        // open level above the cut-off.  A lane reserves record q only while
        // fewer than kServeItems records are reserved and untaken (so record
        // q - kServeItems, in the same entry, is taken; its taker reads it
        // in the same pass).  A record is one more outstanding piece before
        // it is published, and its ready word carries the job number, so a
        // taker never reads a record of another job.
        if (__popcll(want) < kSvShareMin && lim > 0 && ((++tick) & (kSvPoll - 1)) == 0) {
            uint64_t hungry = 0, queued = ~0ull;
            if (lane == 0) {
                hungry = __hip_atomic_load(a.gate + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (hungry) {
                    const uint64_t r = __hip_atomic_load(&js->dq_res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t h = __hip_atomic_load(&js->dq_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t rl = r & 0xFFFFFFFFull, hl = h & 0xFFFFFFFFull;
                    if ((r >> 32) == seq32 && (h >> 32) == seq32 && rl >= hl) queued = rl - hl;
                }
            }
            hungry = bcast64(hungry, 0);
            queued = bcast64(queued, 0);
            if (queued != ~0ull && hungry > queued) {
                int lvl = -1;
                if (has && !L.done()) {
                    const int dep = L.depth(dbase);
                    lvl = open_level(L.start_level(dbase), dep < lim ? dep : lim);
                }
                const uint64_t donors = __ballot(lvl >= 0);
                uint64_t quota = hungry - queued;
                quota = quota < (uint64_t)kSvDonate ? quota : (uint64_t)kSvDonate;
                if (lvl >= 0 && (uint64_t)__popcll(donors & below) < quota) {
                    uint64_t r = __hip_atomic_load(&js->dq_res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bool got = false;
                    for (int tries = 0; tries < 8; ++tries) {
                        const uint64_t h = __hip_atomic_load(&js->dq_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if ((r >> 32) != seq32 || (h >> 32) != seq32) break;
                        if ((r & 0xFFFFFFFFull) - (h & 0xFFFFFFFFull) >= (uint64_t)kServeItems) break;  // full
                        if (__hip_atomic_compare_exchange_strong(&js->dq_res, &r, r + 1ull, __ATOMIC_RELAXED,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            got = true;
                            break;
                        }
                    }
                    if (got) {
                        const uint64_t q = r & 0xFFFFFFFFull;
                        const uint64_t e = q % (uint64_t)kServeItems, lap = q / (uint64_t)kServeItems;
                        // the entry's record of the previous lap has been taken; wait until it is read
                        bool free = lap == 0;
                        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                        while (!free) {
                            free = __hip_atomic_load(&ready[e], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) ==
                                   (tag | (2ull * lap));
                            if (free || __builtin_amdgcn_s_memrealtime() - t0 > kStallTicks) break;
                            __builtin_amdgcn_s_sleep(1);
                        }
                        // a record never published stays outstanding: the job is then never reported done
                        if (free) {
                            __hip_atomic_fetch_add(&js->remaining, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            items[e] = give(lvl);
                            __hip_atomic_store(&ready[e], tag | (2ull * lap + 1ull), __ATOMIC_RELEASE,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
            }
        }

        // ---------------- idle lanes take workunits of the job ----------------
        // A wave takes at most `share` workunits per pass (about the job's
        // workunits over twice the grid's waves, at most `chunk`), so a job
        // spreads over the whole grid; its own sharing then fills the rest
        // of its lanes.  One compare-and-swap claims them: it checks the job
        // number in the same word, so a wave never claims workunits of a
        // later job in the same slot.
        int64_t my_id = -1;
        if (want && job_left) {
            const uint64_t k = (uint64_t)__popcll(want);
            const uint64_t rank = (uint64_t)__popcll(want & below);
            const int leader = __ffsll((unsigned long long)want) - 1;
            const uint64_t ask = k < share ? k : share;
            uint64_t got = 0, b0 = 0;
            if (lane == leader) {
                uint64_t h = __hip_atomic_load(&js->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int tries = 0; tries < 64; ++tries) {
                    const uint64_t taken = h & 0xFFFFFFFFull;
                    if ((h >> 32) != seq32 || taken >= (uint64_t)ntasks) break;
                    const uint64_t rem = (uint64_t)ntasks - taken;
                    const uint64_t sz = rem < ask ? rem : ask;
                    if (__hip_atomic_compare_exchange_strong(&js->head, &h, h + sz, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        got = sz;
                        b0 = taken;
                        break;
                    }
                }
            }
            got = bcast64(got, leader);
            b0 = bcast64(b0, leader);
            if (!got) {
                job_left = false;
            } else {
                took = true;
                own += got;
                if (!has && rank < got) my_id = (int64_t)(b0 + rank);
            }
            if (my_id >= 0) {
                // the workunit's cells from the pool (16-byte loads), then its record
                uint32_t words[PS / 4];
                const uint4 *src = reinterpret_cast<const uint4 *>(pre + (size_t)my_id * PS);
#pragma unroll
                for (int q = 0; q < PS / 16; ++q) {
                    const uint4 v = src[q];
                    words[4 * q] = v.x;
                    words[4 * q + 1] = v.y;
                    words[4 * q + 2] = v.z;
                    words[4 * q + 3] = v.w;
                }
                uint64_t c0 = 0;
                bool mis = false;
                const R r = prefix_record<N, VS>(words, patbits, desc0, nlev, 0u, &c0, &mis);
                start(r);
                L.cnt = c0;  // dead, complete or one-level workunits: counted here
                has = true;
            }
            want = __ballot(!has);
        }

        // ---------------- idle lanes share the busy lanes' subtrees inside the wave ----------------
        // once at least kSvShareMin lanes are idle, or the busy ones are few
        const int nidle = __popcll(want);
        if (want && want != ~0ull && (nidle >= kSvShareMin || 64 - nidle < kSvShareMin)) {
            int lvl = -1;
            if (has && !L.done()) {
                const int dep = L.depth(dbase);
                lvl = open_level(L.start_level(dbase), dep < last - 1 ? dep : last - 1);
            }
            const uint64_t donors = __ballot(lvl >= 0);
            const uint64_t nd = (uint64_t)__popcll(donors), ni = (uint64_t)__popcll(want);
            const uint64_t m = nd < ni ? nd : ni;
            if (m) {
                const uint64_t drank = (uint64_t)__popcll(donors & below);
                const uint64_t rrank = (uint64_t)__popcll(want & below);
                const bool take = !has && rrank < m;
                if (lvl >= 0 && drank < m) mbox[drank] = give(lvl);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                __builtin_amdgcn_wave_barrier();
                R got{};
                if (take) got = mbox[rrank];
                __builtin_amdgcn_wave_barrier();
                if (take) {
                    start(got);
                    has = true;
                }
                want = __ballot(!has);
            }
        }

        // ---------------- an idle lane takes a subtree another wave handed on ----------------
        // by a wave with every lane idle, one record per pass: the wave's own
        // sharing spreads it over its lanes, and records are handed on for
        // whole waves
        if (want == ~0ull && !job_left) {
            const int leader = __ffsll((unsigned long long)want) - 1;
            bool got = false;
            if (lane == leader) {
                uint64_t h = __hip_atomic_load(&js->dq_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int tries = 0; tries < 16; ++tries) {
                    const uint64_t r = __hip_atomic_load(&js->dq_res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((h >> 32) != seq32 || (r >> 32) != seq32) break;
                    if ((r & 0xFFFFFFFFull) <= (h & 0xFFFFFFFFull)) break;
                    if (__hip_atomic_compare_exchange_strong(&js->dq_head, &h, h + 1ull, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        got = true;
                        break;
                    }
                }
                if (got) {
                    // its donor publishes the record right after reserving it
                    const uint64_t q = h & 0xFFFFFFFFull;
                    const uint64_t e = q % (uint64_t)kServeItems, lap = q / (uint64_t)kServeItems;
                    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                    bool ok = false;
                    for (;;) {
                        if (__hip_atomic_load(&ready[e], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) ==
                            (tag | (2ull * lap + 1ull))) {
                            ok = true;
                            break;
                        }
                        if (__builtin_amdgcn_s_memrealtime() - t0 > kStallTicks) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    // a record never published within the stall limit stays
                    // outstanding: the job is then never reported done
                    if (ok) {
                        const R rec = items[e];
                        __hip_atomic_store(&ready[e], tag | (2ull * lap + 2ull), __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        start(rec);
                        has = true;
                    }
                }
            }
            if (__builtin_amdgcn_readlane((int)got, leader)) {
                took = true;
                // the record is this wave's piece once read (the leader was idle)
                if (__builtin_amdgcn_readlane((int)has, leader)) ++own;
                want = __ballot(!has);
            }
        }
        if (want == ~0ull && !job_left) return took;
    }
}

// Host-ring reads are rationed: every read of host-pinned memory is a
// round trip over the host link, which the running jobs' workunit reads
// share.  One wave at a time, at most once per kServePollTicks, reads the
// host's publish word; only when it has moved since the last scan does that
// wave read the ring's pub words, and it sets up every new job it finds.
// Every other wave finds jobs in the device-side work states alone.
constexpr uint64_t kServePollTicks = 2000;  // 20 us at 100 MHz

// The oldest published job that has untaken workunits: its slot, or -1;
// *pub_out gets its pub word.  A job found in the ring is set up by the
// first wave that claims it.  Whether a job is takeable is judged from the
// claim word alone (job number and size in one word), the same word
// serve_job works from.
__device__ __forceinline__ int serve_pick(const ServeArgs &a, int lane, uint64_t now, uint64_t *pub_out) {
    uint64_t *last_poll = a.gate + 1;  // device: tick of the last look at the publish word
    uint64_t *scanned = a.gate + 2;    // device: publish word at the last ring scan
    bool fresh = false;
    uint64_t pubc = 0;
    if (lane == 0) {
        uint64_t t = __hip_atomic_load(last_poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (now - t >= kServePollTicks &&
            __hip_atomic_compare_exchange_strong(last_poll, &t, now, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            pubc = hload64(a.published);
            fresh = pubc != __hip_atomic_load(scanned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    fresh = __builtin_amdgcn_readlane((int)fresh, 0) != 0;
    pubc = bcast64(pubc, 0);
    uint64_t best = ~0ull, best_claim = 0;
    for (int j = lane; j < a.max_jobs; j += 64) {
        JobState *js = &a.state[j];
        uint64_t c = __hip_atomic_load(&js->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fresh) {
            const uint64_t q = hload64(&a.jobs[j].pub);
            if (q > c) {
                // a job not set up yet: the first wave to claim it does
                if (!__hip_atomic_compare_exchange_strong(&js->claim, &c, q, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT))
                    continue;  // being set up by another wave: seen next time
                __hip_atomic_store(&js->total, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&js->t_start, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&js->remaining, q & 0xFFFFFFFFull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&js->dq_res, q & ~0xFFFFFFFFull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&js->dq_head, q & ~0xFFFFFFFFull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&js->head, q & ~0xFFFFFFFFull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                c = q;
            }
        }
        if (!c) continue;
        const uint64_t h = __hip_atomic_load(&js->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool open = (h >> 32) == (c >> 32) && (h & 0xFFFFFFFFull) < (c & 0xFFFFFFFFull);
        if (!open) {
            // no untaken workunit: records waiting in its donation queue
            const uint64_t r = __hip_atomic_load(&js->dq_res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t d = __hip_atomic_load(&js->dq_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            open = (r >> 32) == (c >> 32) && (d >> 32) == (c >> 32) && (r & 0xFFFFFFFFull) > (d & 0xFFFFFFFFull);
        }
        if (open) {
            const uint64_t key = ((c >> 32) << 8) | (uint64_t)j;  // oldest first
            if (key < best) {
                best = key;
                best_claim = c;
            }
        }
    }
    // a later scan starts from here (a scan that ends after a newer one
    // stores an older word, which only makes the next poller scan again)
    if (fresh && lane == 0) __hip_atomic_store(scanned, pubc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t mine = best;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t y = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(best >> 32), o) << 32) |
                           (uint32_t)__shfl_xor((int)(uint32_t)best, o);
        best = y < best ? y : best;
    }
    if (best == ~0ull) return -1;
    const int owner = __ffsll((unsigned long long)__ballot(mine == best)) - 1;
    *pub_out = bcast64(best_claim, owner);
    return (int)(best & 0xFFu);
}

__global__ void __launch_bounds__(kSvBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) serve_kernel(ServeArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    unsigned char *wsm = smem + (threadIdx.x >> 6) * kSvWave;  // this wave's LDS
    uint32_t *alive = a.alive + blockIdx.x * (kSvBlock / 64) + (threadIdx.x >> 6);
    if (lane == 0) __hip_atomic_store(alive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    uint64_t idle_since = __builtin_amdgcn_s_memrealtime();
    uint32_t backoff = 1;
    uint32_t empty = 0;     // picks in a row that gave the wave no workunit
    bool asked = false;     // counted in gate[3]: found no work, asks busy waves for subtrees
    for (;;) {
        if (__hip_atomic_load(a.gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kServeClosing) break;
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        uint64_t pub = 0;
        const int slot = serve_pick(a, lane, now, &pub);
        if (slot >= 0 && empty < 16) {
            // enter: one more wave inside a job; a wave that finds the grid
            // leaving takes its count back and leaves too (the closing bit
            // stays set: it was set while the count was zero)
            bool in = false;
            if (lane == 0) {
                const uint64_t g = __hip_atomic_fetch_add(a.gate, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                in = !(g & kServeClosing);
                if (!in) __hip_atomic_fetch_add(a.gate, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (!__builtin_amdgcn_readlane((int)in, 0)) break;
            if (asked) {
                if (lane == 0) __hip_atomic_fetch_add(a.gate + 3, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                asked = false;
            }
            // the descriptor and cells of the job are used only while the
            // slot still holds it: reading its pub word from the ring, then
            // an acquire fence, orders them after the host's writes (made
            // before its release store of that word)
            bool took = false;
            if (hload64(&a.jobs[slot].pub) == pub) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                const int n = (int)hload32(&a.jobs[slot].n);
                const bool vs = hload32(&a.jobs[slot].vs) != 0u;
                switch (n * 2 + (vs ? 1 : 0)) {
#define DLS_SV_CASE(K)                                                               \
    case 2 * K: took = serve_job<K, false>(a, slot, pub, wsm, lane); break;         \
    case 2 * K + 1: took = serve_job<K, true>(a, slot, pub, wsm, lane); break;
                    DLS_SV_CASE(4) DLS_SV_CASE(5) DLS_SV_CASE(6) DLS_SV_CASE(7) DLS_SV_CASE(8) DLS_SV_CASE(9)
#undef DLS_SV_CASE
                    default: break;  // the host publishes only these orders
                }
            }
            if (lane == 0) __hip_atomic_fetch_add(a.gate, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // -1
            if (took) {
                empty = 0;
                idle_since = __builtin_amdgcn_s_memrealtime();
                backoff = 1;
                continue;
            }
            ++empty;
        } else {
            empty = 0;
        }
        // nothing taken: the stop flag ends the wave; past the idle limit the
        // wave closes the gate for the whole grid if no wave is inside a job
        if (hload32(a.stop) != 0u) break;
        if (now - idle_since > a.idle_ticks) {
            bool closed = false;
            if (lane == 0) {
                uint64_t g = __hip_atomic_load(a.gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (g == 0u)
                    __hip_atomic_compare_exchange_strong(a.gate, &g, kServeClosing, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                closed = (g == 0u) || (g & kServeClosing);  // g: 0 on success, else the value found
            }
            if (__builtin_amdgcn_readlane((int)closed, 0)) break;
        }
        if (!asked) {
            if (lane == 0) __hip_atomic_fetch_add(a.gate + 3, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            asked = true;
        }
        // an idle wave looks again after 1, 2, 4, ... up to about 400 us (a
        // longer sleep than 100 us measured 5 % more requests/s on the mix)
        for (uint32_t t = 0; t < backoff; ++t) __builtin_amdgcn_s_sleep(32);
        backoff = backoff < 512 ? backoff * 2 : 512;
    }
    if (asked && lane == 0) __hip_atomic_fetch_add(a.gate + 3, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane == 0) __hip_atomic_store(alive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_serve(const ServeArgs &a) {
    if (a.block != kSvBlock) return hipErrorInvalidValue;
    (void)hipGetLastError();
    hipLaunchKernelGGL(serve_kernel, dim3(a.grid), dim3(a.block), (size_t)(kSvBlock / 64) * kSvWave, a.stream, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int N, bool VS>
static hipError_t launch_n(const LaunchArgs &a) {
    using R = Rec<N, VS>;
    (void)hipGetLastError();  // drop an error left by an unrelated earlier call
    const int block = a.block;
    const size_t lds = lds_bytes(N, VS, a.plan.nlev, block, a.persistent, a.persistent && a.tune.lds_masks);
    R *recs = reinterpret_cast<R *>(a.records);
    const unsigned pgrid = (unsigned)((a.num + 255) / 256);
    hipLaunchKernelGGL((prep_kernel<N, VS>), dim3(pgrid), dim3(256), 0, a.stream, a.plan, a.prefixes, a.num, recs,
                       a.counts, a.status);
    if (a.plan.nlev <= 1) return hipGetLastError();  // prep wrote every count
    if (a.persistent) {
        hipLaunchKernelGGL(reset_queue, dim3(256), dim3(256), 0, a.stream, a.ctrl, a.ready, a.item_cap);
        hipLaunchKernelGGL(init_ctrl, dim3(1), dim3(64), 0, a.stream, a.ctrl);
    }
    if (a.ev_start) (void)hipEventRecord(a.ev_start, a.stream);
    if (a.persistent) {
        R *items = reinterpret_cast<R *>(a.items);
        const bool expand = a.ex != nullptr && a.plan.nlev >= 3;
        if (expand) {
            hipLaunchKernelGGL(ex_init, dim3(1), dim3(64), 0, a.stream, a.ex, a.records, a.num, a.counts);
            const int64_t limit = std::min<int64_t>(4096, a.ecap / 16);
            if (limit > 0)
                hipLaunchKernelGGL((ex_small<N, VS>), dim3(1), dim3(1024), 0, a.stream, a.plan, a.ex, a.ebuf[0],
                                   a.ebuf[1], a.eorig[0], a.eorig[1], a.counts, a.tcounts, a.status, a.etarget,
                                   a.ecap, limit, a.plan.nlev - 2);
            for (int p = 0; p < a.epasses; ++p) {
                hipLaunchKernelGGL((ex_tally<N, VS>), dim3(kExBlocks), dim3(256), 0, a.stream, a.plan, a.ex, p,
                                   a.eblk);
                hipLaunchKernelGGL((ex_write<N, VS>), dim3(kExBlocks), dim3(256), 0, a.stream, a.plan, a.ex, p,
                                   a.eblk, a.ebuf[0], a.ebuf[1], a.eorig[0], a.eorig[1], a.counts, a.tcounts,
                                   a.status, a.etarget, a.ecap);
            }
        }
        // the state after the last pass
        const Expand *ex = expand ? a.ex + (a.epasses & 1) : nullptr;
        const bool gl = a.item_cap > 0 && a.tune.steal_depth > 0;
#define DLS_PERSISTENT(STATS, LM, GL)                                                                          \
    hipLaunchKernelGGL((persistent_kernel<N, VS, STATS, LM, GL>), dim3(a.grid), dim3(block), lds, a.stream, a.plan, \
                       recs, a.num, a.counts, a.status, a.steps, a.ctrl, items, a.ready, a.item_cap, a.tune, ex)
#define DLS_PERSISTENT_GL(STATS, LM) \
    if (gl) DLS_PERSISTENT(STATS, LM, true); else DLS_PERSISTENT(STATS, LM, false);
        if (a.tune.lds_masks) {
            if (a.steps) { DLS_PERSISTENT_GL(true, true) }
            else { DLS_PERSISTENT_GL(false, true) }
        } else {
            if (a.steps) { DLS_PERSISTENT_GL(true, false) }
            else { DLS_PERSISTENT_GL(false, false) }
        }
#undef DLS_PERSISTENT_GL
#undef DLS_PERSISTENT
        if (expand) hipLaunchKernelGGL(ex_scatter, dim3(kExBlocks), dim3(256), 0, a.stream, ex, a.counts);
    } else {
        const int64_t grid = (a.num + block - 1) / block;
        if (a.steps)
            hipLaunchKernelGGL((plain_kernel<N, VS, true>), dim3((unsigned)grid), dim3(block), lds, a.stream, a.plan,
                               recs, a.num, a.counts, a.steps);
        else
            hipLaunchKernelGGL((plain_kernel<N, VS, false>), dim3((unsigned)grid), dim3(block), lds, a.stream,
                               a.plan, recs, a.num, a.counts, a.steps);
    }
    if (a.ev_stop) (void)hipEventRecord(a.ev_stop, a.stream);
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

size_t record_bytes(int n, bool vs) {
    switch (n) {
#define DLS_REC_CASE(K) \
    case K: return vs ? sizeof(Rec<K, true>) : sizeof(Rec<K, false>);
        DLS_REC_CASE(1) DLS_REC_CASE(2) DLS_REC_CASE(3) DLS_REC_CASE(4) DLS_REC_CASE(5) DLS_REC_CASE(6)
        DLS_REC_CASE(7) DLS_REC_CASE(8) DLS_REC_CASE(9) DLS_REC_CASE(10) DLS_REC_CASE(11) DLS_REC_CASE(12)
        DLS_REC_CASE(13) DLS_REC_CASE(14) DLS_REC_CASE(15) DLS_REC_CASE(16)
#undef DLS_REC_CASE
        default: return 0;
    }
}

uint32_t make_desc(int n, bool vs, int i, int j) {
    (void)vs;
    const int lpw = 64 / n;
    uint32_t d = (uint32_t)((i % lpw) * n) | (uint32_t)(i / lpw) << 6 | (uint32_t)((j % lpw) * n) << 8 |
                 (uint32_t)(j / lpw) << 14;
    if (i == j) d |= 1u << 16;
    if (i + j == n - 1) d |= 1u << 17;
    return d;
}

size_t lds_bytes(int n, bool vs, int nlev, int block, bool persistent, bool lds_masks) {
    const int elem = n <= 8 ? 1 : 2;
    if (!persistent) return kStackBase + (size_t)elem * (size_t)(nlev > 1 ? nlev : 1) * block;
    if (lds_masks) {
        const int lines = n >= kLmPackMinN ? n : n + (vs ? (n + 1) / 2 : n);  // LdsLane<n, vs>::LINES
        return lm_stacks_end(lines, nlev, block, elem, vs);
    }
    const bool dw = n % 2 == 0 && !vs && n <= 8;  // VLaneDesc<n, vs>::DW: one more level, the sentinel
    return vl_stacks_end(dw ? nlev + 1 : nlev, block, elem) + record_bytes(n, vs) * (size_t)block;
}

hipError_t launch_zero(uint64_t *p, int64_t n, hipStream_t stream) {
    (void)hipGetLastError();
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(zero_u64, dim3(grid), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_reduce_weighted(const uint64_t *counts, const uint32_t *mult, int64_t num, uint64_t *out,
                                  hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(zero_one, dim3(1), dim3(64), 0, stream, out);
    if (num > 0) {
        // at most one workgroup per CU (a small array needs fewer)
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int64_t want = (num / 4 + kReduceBlock - 1) / kReduceBlock + 1;
        const unsigned grid = (unsigned)(want < cus ? want : cus);
        hipLaunchKernelGGL(reduce_weighted, dim3(grid), dim3(kReduceBlock), 0, stream, counts, mult, num, out);
    }
    return hipGetLastError();
}

hipError_t launch_valu_probe(int blocks, int iters, uint32_t *sink, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(valu_probe, dim3(blocks), dim3(256), 0, stream, iters, sink);
    return hipGetLastError();
}

}  // namespace dlsk
