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
    kErrCbInfeasible = 1u << 8, // device codebook: more used symbols than 2^L codewords
    kErrCbTooMany = 1u << 9,    // device codebook: more used symbols than one workgroup ranks
    kErrCbCount = 1u << 10,     // device codebook: a count of 2^40 or more
};

// Library-internal decode calls for the serving loop (C++ linkage, not part
// of the C ABI).  Their status goes to a caller-zeroed word, typically in
// pinned host memory: a wavefront that met an error stores its nonzero bits
// there with a plain store (bits of different wavefronts may overwrite one
// another; the word is nonzero exactly when some wavefront erred), so no
// status copy follows the decode.
//   decode_gap_direct: hd_decode in HD_MODE_GAP without a workspace (one
//     kernel launch);
//   decode_batch_direct: hd_decode_batch with its status word replaced.
hd_status decode_gap_direct(const hd_dstream *s, uint16_t *out, uint32_t *status_word, void *hip_stream);
hd_status decode_batch_direct(const hd_dstream *streams, uint32_t n_streams, uint16_t *const *outs,
                              uint32_t *status_word, void *workspace, size_t ws_bytes, void *hip_stream);

constexpr uint32_t kLenLong = 0;     // first-level entry: codeword longer than lut_bits
constexpr uint32_t kLenBad = 63;     // first-level entry: prefix of no codeword

}  // namespace hd
