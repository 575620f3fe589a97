// dls_canon.hip -- hourglass designs and their canonical forms on the GPU
// (Sec. 4.2-4.3, Alg. 5).
//
// Input: diagonal designs (first row, main diagonal and antidiagonal assigned,
// nothing else), one lane each.  The lane enumerates every consistent filling
// of the free cells of the last row (the corners lie on the diagonals), so
// each leaf is an hourglass design, and tests it for canonicity under the
// hourglass transformation group: for every element g the image of the
// design's known cells is renamed so that its first row reads 0..n-1 and
// compared with the design in row-major order over the hourglass cells; the
// design is canonical when no image is smaller, and its class power is
// |G| / (number of elements whose image equals it).  Canonical designs are
// appended to the output with their class power.
//
// The group comes in as a table src[g][k]: the hourglass cell (index into
// the row-major list of hourglass cells) whose value lands on hourglass cell
// k under g.  Table and per-lane designs live in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dls_canon.hpp"

namespace dlsc {

size_t canon_lds_bytes(int n, int groups, int kcells) {
    return (size_t)((groups * kcells + 15) & ~15) + (size_t)((kcells + 15) & ~15) +
           256u * (size_t)(((kcells + 3) & ~3) + 4 * n);
}

namespace {

template <int N>
__global__ void __launch_bounds__(256) canon_kernel(const uint8_t *__restrict__ designs, int64_t num,
                                                    const uint8_t *__restrict__ src_tab, int groups, int kcells,
                                                    const uint8_t *__restrict__ hc, uint8_t *out, uint32_t *out_mult,
                                                    int64_t cap, unsigned long long *out_count, uint32_t *status) {
    constexpr int NN = N * N;
    constexpr uint32_t ALL = (1u << N) - 1u;
    extern __shared__ __align__(16) unsigned char smem[];
    uint8_t *tab = smem;                                     // groups * kcells
    const int tab_bytes = (groups * kcells + 15) & ~15;
    uint8_t *hcs = smem + tab_bytes;                         // kcells flat cell indices
    // per lane: its design's hourglass values, then the DFS candidate sets and
    // the column masks of the last row (16 bits each)
    const int lane_bytes = ((kcells + 3) & ~3) + 4 * N;
    uint8_t *mine = hcs + ((kcells + 15) & ~15) + threadIdx.x * lane_bytes;
    uint16_t *cand = reinterpret_cast<uint16_t *>(mine + ((kcells + 3) & ~3));
    uint16_t *colmask = cand + N;
    for (int t = threadIdx.x; t < groups * kcells; t += blockDim.x) tab[t] = src_tab[t];
    for (int t = threadIdx.x; t < kcells; t += blockDim.x) hcs[t] = hc[t];
    __syncthreads();

    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= num) return;
    const uint8_t *d = designs + idx * NN;
    // hourglass cell values of the design (last row: corners only, so far)
    for (int k = 0; k < kcells; ++k) mine[k] = d[hcs[k]];
    // free cells of the last row: hourglass positions kcells-n+1 .. kcells-2
    const int k0 = kcells - N;
    uint32_t rowmask = 0;
    for (int j = 0; j < N; ++j) colmask[j] = 0;
    for (int c = 0; c < NN - N; ++c) {
        const uint32_t v = d[c];
        if (v < (uint32_t)N) colmask[c % N] = (uint16_t)(colmask[c % N] | (1u << v));
    }
    {
        const uint32_t a = d[NN - N], b = d[NN - 1];
        if (a >= (uint32_t)N || b >= (uint32_t)N || a == b || (colmask[0] >> a & 1u) || (colmask[N - 1] >> b & 1u))
            return;  // not a consistent diagonal design
        rowmask = (1u << a) | (1u << b);
    }
    // iterative DFS over the last row's free cells j = 1 .. n-2
    int j = 1;
    cand[1] = (uint16_t)(ALL & ~(rowmask | colmask[1]));
    for (;;) {
        const uint32_t cj = cand[j];
        if (cj == 0u) {
            if (j == 1) break;
            --j;
            const uint32_t v = mine[k0 + j];
            rowmask ^= 1u << v;
            continue;
        }
        const uint32_t b = cj & (0u - cj);
        cand[j] = (uint16_t)(cj ^ b);
        const uint32_t v = (uint32_t)__builtin_ctz(b);
        mine[k0 + j] = (uint8_t)v;
        if (j < N - 2) {
            rowmask |= b;
            ++j;
            cand[j] = (uint16_t)(ALL & ~(rowmask | colmask[j]));
            continue;
        }
        // a complete hourglass design: canonicity test (Alg. 5)
        int stab = 0;
        bool canonical = true;
        for (int g = 0; g < groups && canonical; ++g) {
            const uint8_t *s = tab + g * kcells;
            uint64_t sig = 0;  // renaming: value -> position in the image's first row
            for (int t = 0; t < N; ++t) sig |= (uint64_t)t << (4 * mine[s[t]]);
            int cmp = 0;
            for (int k = N; k < kcells; ++k) {
                const uint32_t img = (uint32_t)(sig >> (4 * mine[s[k]])) & 15u, own = mine[k];
                if (img != own) {
                    cmp = img < own ? -1 : 1;
                    break;
                }
            }
            if (cmp < 0) canonical = false;
            stab += cmp == 0;
        }
        if (canonical) {
            const unsigned long long slot = atomicAdd(out_count, 1ull);
            if (slot < (unsigned long long)cap) {
                uint8_t *o = out + slot * NN;
                for (int c = 0; c < NN; ++c) o[c] = d[c];
                for (int t = 1; t < N - 1; ++t) o[NN - N + t] = mine[k0 + t];
                out_mult[slot] = (uint32_t)(groups / stab);
            } else if (status) {
                atomicOr(status, 8u);
            }
        }
    }
}

template <int N>
hipError_t launch_n(const CanonArgs &a) {
    const size_t lds = canon_lds_bytes(N, a.groups, a.kcells);
    const unsigned grid = (unsigned)((a.num + 255) / 256);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((canon_kernel<N>), dim3(grid), dim3(256), lds, a.stream, a.designs, a.num, a.src_tab, a.groups,
                       a.kcells, a.hc, a.out, a.out_mult, a.cap, a.out_count, a.status);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_canon(const CanonArgs &a) {
    (void)hipGetLastError();
    switch (a.n) {
        case 4: return launch_n<4>(a);
        case 5: return launch_n<5>(a);
        case 6: return launch_n<6>(a);
        case 7: return launch_n<7>(a);
        case 8: return launch_n<8>(a);
        case 9: return launch_n<9>(a);
        case 10: return launch_n<10>(a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dlsc
