// dms_common.hpp -- shared device helpers and host argument checks.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dms.h"

namespace dms {

constexpr int kWave = 64;

// ---------------------------------------------------------------- host side

inline bool box_valid(const int64_t *dims, const int64_t *lo, const int64_t *hi)
{
    if (!dims || !lo || !hi) return false;
    for (int c = 0; c < 3; ++c) {
        if (dims[c] < 1) return false;
        if (lo[c] < 0 || hi[c] > dims[c] || lo[c] > hi[c]) return false;
    }
    return true;
}

inline bool grid_size_ok(const int64_t *dims)
{
    // int32 orders rank at most 2^31 - 1 vertices, and INT32_MAX is reserved
    // as the "absent neighbour" sentinel.
    const int64_t lim = 2147483647LL;
    if (dims[0] > lim || dims[1] > lim || dims[2] > lim) return false;
    if (dims[0] * dims[1] > lim) return false;
    return dims[0] * dims[1] * dims[2] <= lim;
}

// Grids that need no int32 order (the gradient from the values, the
// extraction): each side below 2^31, at most 2^40 vertices (record indices in
// the gradient queue take 40 bits; cell codes (vertex << 8) stay far inside
// int64).
inline bool grid_size_values_ok(const int64_t *dims)
{
    const int64_t lim = 2147483647LL;
    if (dims[0] > lim || dims[1] > lim || dims[2] > lim) return false;
    const int64_t plane = dims[0] * dims[1];
    if (plane > (1LL << 40)) return false;
    return dims[2] <= (1LL << 40) / plane;
}

// DMS_OK when the current device is a gfx950 (its properties are read once
// per device and remembered), else DMS_E_UNSUPPORTED (also without a device).
int device_check();

inline int launch_status()
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DMS_OK : DMS_E_HIP;
}

constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// -------------------------------------------------------------- device side

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Order-preserving unsigned keys (Section 2.1 compares values; -0.0 equals
// +0.0).  The sign bit selects between flipping all bits (negative values)
// and flipping only the sign bit (positive values), after mapping -0.0 to
// +0.0.  NaN inputs are reported through the flag word.
__device__ __forceinline__ uint32_t key_of(float v, bool &nan)
{
    uint32_t b = __float_as_uint(v);
    if (b == 0x80000000u) b = 0u;
    nan = (b & 0x7fffffffu) > 0x7f800000u;
    return b ^ ((b & 0x80000000u) ? 0xffffffffu : 0x80000000u);
}

// Unsigned 64-bit integers are their own keys (used to sort composite
// integer keys with the same passes).
__device__ __forceinline__ uint64_t key_of(uint64_t v, bool &nan)
{
    nan = false;
    return v;
}

__device__ __forceinline__ uint64_t key_of(double v, bool &nan)
{
    uint64_t b = (uint64_t)__double_as_longlong(v);
    if (b == 0x8000000000000000ull) b = 0ull;
    nan = (b & 0x7fffffffffffffffull) > 0x7ff0000000000000ull;
    return b ^ ((b & 0x8000000000000000ull) ? 0xffffffffffffffffull : 0x8000000000000000ull);
}

// Lanes of the wave (among `active`) holding the same 8-bit digit as this
// lane: intersect, bit by bit, the ballot of lanes agreeing with it.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t active)
{
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

}  // namespace dms
