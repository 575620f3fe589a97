// dls_canon.hpp -- launch interface of the hourglass canonicalisation kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dlsc {

struct CanonArgs {
    int n;
    const uint8_t *designs;         // num diagonal designs, n*n bytes each (device)
    int64_t num;
    const uint8_t *src_tab;         // groups * kcells (device)
    int groups;
    int kcells;
    const uint8_t *hc;              // kcells flat indices of the hourglass cells, row-major (device)
    uint8_t *out;                   // cap canonical designs, n*n bytes each (device)
    uint32_t *out_mult;             // cap class powers (device)
    int64_t cap;
    unsigned long long *out_count;  // designs found (may exceed cap) (device, caller-zeroed)
    uint32_t *status;               // bit 3: output capacity exceeded (device, may be null)
    hipStream_t stream;
};

// LDS bytes per workgroup of 256 lanes.
size_t canon_lds_bytes(int n, int groups, int kcells);
hipError_t launch_canon(const CanonArgs &a);

}  // namespace dlsc
