// Declarations shared by the host and device translation units of the library.
#pragma once

#include <cstdint>

#include "hd.h"

extern "C" {
// Canonical codes from code lengths (hd_host.cpp).  HD_ERR_ARG when the
// lengths oversubscribe the code space or exceed L.
hd_status hd_canonical_codes_internal(const uint8_t *len, uint32_t A, uint32_t L, uint32_t *codes);
}

namespace hd {

// Status bits OR-ed into the workspace status word by the kernels.
enum : uint32_t {
    kErrGapRange = 1u << 0,     // a gap byte larger than any codeword allows
    kErrBadCode = 1u << 1,      // a window matched no codeword
    kErrLaneEnd = 1u << 2,      // a subsequence ended off its successor's start
    kErrChunkSum = 1u << 3,     // decoded count of a chunk != its stored offsets
    kErrTotal = 1u << 4,        // chunk offsets not from 0 to n_symbols (self-sync: totals)
    kErrOutRange = 1u << 5,     // an output index fell outside [0, n)
    kErrNoSync = 1u << 6,       // the synchronized path does not end on the stream end
    kErrNoOutlier = 1u << 7,    // reconstruction: a code-0 position missing from the outlier list
};

constexpr uint32_t kLenLong = 0;     // first-level entry: codeword longer than lut_bits
constexpr uint32_t kLenBad = 63;     // first-level entry: prefix of no codeword

}  // namespace hd
