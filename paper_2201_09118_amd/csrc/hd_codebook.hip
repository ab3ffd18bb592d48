// Codebook construction on the device (gfx950): the optimal length-limited
// code lengths and canonical codes of hd_build_codebook, from a histogram in
// device memory, so that a device encode needs no host round trip.  The
// paper takes its codebook from the cuSZ encoder, whose GPU codebook builder
// it cites (Sec. II-B, Sec. VI); the construction here is the library's own
// package-merge (counting form) with the same tie rule as the host builder,
// so both give the same bytes.
//
// One workgroup of 1024 work-items does the whole build in LDS:
//   1. the used symbols are gathered (any order) as 64-bit keys
//      count << 24 | symbol, and bitonic-sorted: the ranking by
//      (count, symbol);
//   2. level L is the ranked symbols; for d = L-1 .. 1, level d merges the
//      symbols with the pairs of consecutive items of level d+1 (a symbol
//      ahead of a pair of equal weight).  Each work-item takes a range of
//      output pairs, finds where the range starts in both inputs by a binary
//      search along the merge diagonal, then merges sequentially, summing
//      the next level's pairs as it goes.  For every even prefix 2k of level
//      d it records how many of those items are pairs (global workspace);
//   3. the selection (first 2m-2 items of level 1, then the first 2p items
//      of level d+1 for the p pairs taken at level d) reads one recorded
//      count per level; the symbols taken at level d are the first
//      (taken - pairs) of the ranking, and a symbol's length is the number of
//      levels that take it;
//   4. canonical codes: per-length counts give each length's first code; a
//      symbol's code adds its rank among same-length symbols in symbol
//      order, from wavefront ballots over 1024-symbol chunks.
// Limits: alphabets up to 65536, at most 4096 used symbols, counts below
// 2^40; a histogram outside them (or needing more than 2^L codewords) sets a
// status bit and yields an all-zero codebook.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hd.h"
#include "hd_internal.h"

using namespace hd;

namespace {

constexpr uint32_t kCbThreads = 1024;
constexpr uint32_t kCbMaxUsed = 4096;          // used symbols one workgroup ranks in LDS
constexpr uint32_t kCbMaxAlphabet = 65536;     // the length map lives in LDS
constexpr size_t kCbHead = 256;                // status header (word 0 bits, word 1 = 0)
// prefix counts per level: for k = 0 .. (m + pairs) / 2, the pairs among the
// first 2k items of the level
constexpr size_t kCbLevelWords = kCbMaxUsed + 2;

constexpr size_t cb_ws_bytes(uint32_t L) { return kCbHead + size_t(L + 1) * kCbLevelWords * 4; }

// LDS: sorted keys (32 KB) + two pair buffers (2 x 32 KB, later the 64 KB
// length map) + the per-level pair counts as uint16 when they fit (56 KB:
// (L + 1) (m + 2) entries; larger codes keep them in the global workspace)
// + small counters.
constexpr size_t kCbKeysBytes = size_t(kCbMaxUsed) * 8;
constexpr size_t kCbPairBytes = size_t(kCbMaxUsed) * 8;
constexpr size_t kCbLevelLdsBytes = 56 * 1024;
constexpr size_t kCbLdsBytes = kCbKeysBytes + 2 * kCbPairBytes + kCbLevelLdsBytes;

struct CbShared {
    uint32_t n_used;
    uint32_t flags;
    uint32_t singles[33];      // symbols taken at level d (d = 1 .. L)
    uint32_t bl[34];           // codewords per length
    uint32_t first[34];        // first canonical code per length
    uint32_t base[34];         // codes of each length handed out in earlier chunks
    uint32_t wcnt[16][34];     // per wavefront and length, then its exclusive offset
};

__device__ __forceinline__ uint64_t lane_mask_lt(uint32_t lane)
{
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Items of the merge of A = w(keys[0 .. m)) (the ranked symbols' counts)
// and B = pairs[0 .. nb), a symbol before a pair of equal weight.  Returns
// how many of the first r items are symbols.
__device__ __forceinline__ uint32_t merge_split(const uint64_t *keys, uint32_t m, const uint64_t *pairs,
                                                uint32_t nb, uint32_t r)
{
    uint32_t lo = r > nb ? r - nb : 0u, hi = r < m ? r : m;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        // symbol mid ahead of pair r - mid - 1: more symbols are among the first r
        if ((keys[mid] >> 24) <= pairs[r - mid - 1])
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kCbThreads) void k_codebook(const uint64_t *__restrict__ hist, uint32_t A, uint32_t L,
                                                         uint8_t *__restrict__ len_out,
                                                         uint32_t *__restrict__ code_out, uint32_t *status,
                                                         uint32_t *__restrict__ levels)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ CbShared sh;
    uint64_t *keys = reinterpret_cast<uint64_t *>(smem);
    uint64_t *const pb0 = reinterpret_cast<uint64_t *>(smem + kCbKeysBytes);
    uint64_t *const pb1 = reinterpret_cast<uint64_t *>(smem + kCbKeysBytes + kCbPairBytes);
    uint8_t *lmap = smem + kCbKeysBytes;                  // after the levels: length per symbol
    uint16_t *lev16 = reinterpret_cast<uint16_t *>(smem + kCbKeysBytes + 2 * kCbPairBytes);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;

    if (tid == 0) {
        sh.n_used = 0;
        sh.flags = 0;
    }
    __syncthreads();
    // 1. gather the used symbols
    for (uint32_t s = tid; s < A; s += kCbThreads) {
        const uint64_t w = hist[s];
        if (w) {
            if (w >> 40)
                atomicOr(&sh.flags, kErrCbCount);
            const uint32_t i = atomicAdd(&sh.n_used, 1u);
            if (i < kCbMaxUsed)
                keys[i] = (w << 24) | s;
        }
    }
    __syncthreads();
    const uint32_t m = sh.n_used;
    if (tid == 0) {
        if (m > kCbMaxUsed)
            sh.flags |= kErrCbTooMany;
        if (L < 32 && m > (1u << L))
            sh.flags |= kErrCbInfeasible;
    }
    __syncthreads();
    const uint32_t flags = sh.flags;
    if (flags || m <= 1) {
        // an empty code, a lone symbol (length 1, code 0), or an error (all zero)
        for (uint32_t s = tid; s < A; s += kCbThreads) {
            const bool lone = !flags && m == 1 && hist[s] != 0;
            len_out[s] = lone ? 1 : 0;
            code_out[s] = 0;
        }
        if (tid == 0) {
            status[0] = flags;
            status[1] = 0;
        }
        return;
    }

    // ranking: bitonic sort of the keys, padded to a power of two
    uint32_t N = 2;
    while (N < m)
        N <<= 1;
    for (uint32_t i = m + tid; i < N; i += kCbThreads)
        keys[i] = ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < N; i += kCbThreads) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const uint64_t a = keys[i], b = keys[p];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        keys[i] = b;
                        keys[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }

    // 2. levels.  The pair counts of level d go to lev16[d * (m + 2) ...] when
    // every level fits (one LDS read per level in the selection below),
    // else to the global workspace.
    const uint32_t lstride = m + 2;
    const bool lev_in_lds = size_t(L + 1) * lstride * 2 <= kCbLevelLdsBytes;
    // Pairs of level L (the ranked symbols themselves):
    uint32_t np = m >> 1;
    for (uint32_t k = tid; k < np; k += kCbThreads)
        pb0[k] = (keys[2 * k] >> 24) + (keys[2 * k + 1] >> 24);
    __syncthreads();
    uint32_t cur = 0;
    for (uint32_t d = L - 1; d >= 1; --d) {
        // level d = merge(symbols, the current pair buffer [0 .. np)); its pairs go to the
        // other buffer (not needed after level 1)
        const uint64_t *P = cur ? pb1 : pb0;
        uint64_t *Q = cur ? pb0 : pb1;
        uint32_t *pp = levels + size_t(d) * kCbLevelWords;
        uint16_t *pl = lev16 + size_t(d) * lstride;
        const uint32_t T = m + np;                      // items of level d
        const uint32_t slots = (T + 1) >> 1;            // pair slots (the last may hold one item)
        const uint32_t per = (slots + kCbThreads - 1) / kCbThreads;
        const uint32_t k0 = tid * per, k1 = min(slots, k0 + per);
        if (k0 < k1) {
            uint32_t i = merge_split(keys, m, P, np, 2 * k0);
            uint32_t j = 2 * k0 - i;
            for (uint32_t k = k0; k < k1; ++k) {
                if (lev_in_lds)                         // pairs among the first 2k items
                    pl[k] = static_cast<uint16_t>(j);
                else
                    pp[k] = j;
                uint64_t v[2] = {0, 0};
                for (uint32_t h = 0; h < 2 && 2 * k + h < T; ++h) {
                    if (i < m && (j >= np || (keys[i] >> 24) <= P[j]))
                        v[h] = keys[i++] >> 24;
                    else
                        v[h] = P[j++];
                }
                if (2 * k + 1 < T && d > 1)
                    Q[k] = v[0] + v[1];
            }
        }
        if (tid == 0 && (T & 1u) == 0) {                // the whole level
            if (lev_in_lds)
                pl[T >> 1] = static_cast<uint16_t>(np);
            else
                pp[T >> 1] = np;
        }
        np = T >> 1;
        cur ^= 1;
        __syncthreads();
        if (d == 1)
            break;
    }

    // 3. selection: 2m - 2 items of level 1, then twice the pairs taken
    if (tid == 0) {
        uint32_t take = 2 * m - 2;
        for (uint32_t d = 1; d <= L; ++d) {
            if (d == L) {
                sh.singles[d] = take;                   // level L holds symbols only
                break;
            }
            const uint32_t pairs = lev_in_lds ? lev16[size_t(d) * lstride + (take >> 1)]
                                              : __builtin_nontemporal_load(levels + size_t(d) * kCbLevelWords +
                                                                           (take >> 1));
            sh.singles[d] = take - pairs;
            take = 2 * pairs;
            if (take == 0) {
                for (uint32_t e = d + 1; e <= L; ++e)
                    sh.singles[e] = 0;
                break;
            }
        }
        for (uint32_t l = 0; l < 34; ++l)
            sh.bl[l] = 0;
    }
    // length map cleared (it overlays the pair buffers, free now)
    for (uint32_t s = tid; s < kCbMaxAlphabet / 4; s += kCbThreads)
        reinterpret_cast<uint32_t *>(lmap)[s] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < m; i += kCbThreads) {
        uint32_t depth = 0;
        for (uint32_t d = 1; d <= L; ++d)
            depth += i < sh.singles[d] ? 1u : 0u;
        lmap[keys[i] & 0xffffffu] = static_cast<uint8_t>(depth);
        atomicAdd(&sh.bl[depth], 1u);
    }
    __syncthreads();
    // 4. canonical codes: first code per length as in the host builder
    if (tid == 0) {
        uint32_t c = 0;
        sh.bl[0] = 0;
        for (uint32_t l = 1; l <= 32; ++l) {
            c = (c + sh.bl[l - 1]) << 1;
            sh.first[l] = c;
        }
    }
    if (tid < 34)
        sh.base[tid] = 0;
    for (uint32_t c0 = 0; c0 < A; c0 += kCbThreads) {
        for (uint32_t q = tid; q < 16 * 34; q += kCbThreads)
            (&sh.wcnt[0][0])[q] = 0;
        __syncthreads();
        const uint32_t s = c0 + tid;
        const uint32_t l = s < A ? lmap[s] : 0u;
        uint64_t act = __builtin_amdgcn_ballot_w64(l != 0);
        uint32_t rank = 0;
        while (act) {
            const uint32_t leader = static_cast<uint32_t>(__builtin_ctzll(act));
            const uint32_t ll = static_cast<uint32_t>(__shfl(static_cast<int>(l), static_cast<int>(leader), 64));
            const uint64_t same = __builtin_amdgcn_ballot_w64(l == ll);
            if (l == ll)
                rank = static_cast<uint32_t>(__builtin_popcountll(same & lane_mask_lt(lane)));
            if (lane == 0)
                sh.wcnt[wv][ll] = static_cast<uint32_t>(__builtin_popcountll(same));
            act &= ~same;
        }
        __syncthreads();
        if (tid >= 1 && tid <= 32) {
            uint32_t acc = sh.base[tid];
            for (uint32_t w = 0; w < kCbThreads / 64; ++w) {
                const uint32_t t = sh.wcnt[w][tid];
                sh.wcnt[w][tid] = acc;
                acc += t;
            }
            sh.base[tid] = acc;
        }
        __syncthreads();
        if (s < A) {
            len_out[s] = static_cast<uint8_t>(l);
            code_out[s] = l ? sh.first[l] + sh.wcnt[wv][l] + rank : 0u;
        }
        __syncthreads();
    }
    if (tid == 0) {
        status[0] = 0;
        status[1] = 0;
    }
}

}  // namespace

extern "C" size_t hd_codebook_workspace_size(uint32_t L)
{
    if (L == 0 || L > 32)
        return 0;
    return cb_ws_bytes(L);
}

extern "C" hd_status hd_build_codebook_device(const uint64_t *hist, uint32_t A, uint32_t L, uint8_t *lengths,
                                              uint32_t *codes, void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!hist || !lengths || !codes || !workspace || A == 0 || L == 0 || L > 32)
        return HD_ERR_ARG;
    if (A > kCbMaxAlphabet)
        return HD_ERR_UNSUPPORTED;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 || ws_bytes < cb_ws_bytes(L) ||
        reinterpret_cast<uintptr_t>(hist) % 8 || reinterpret_cast<uintptr_t>(codes) % 4)
        return HD_ERR_ARG;
    static bool lds_ok = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_codebook),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(kCbLdsBytes)) == hipSuccess;
    if (!lds_ok)
        return HD_ERR_DEVICE;
    char *ws = static_cast<char *>(workspace);
    hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kCbThreads), kCbLdsBytes, static_cast<hipStream_t>(hip_stream),
                       hist, A, L, lengths, codes, reinterpret_cast<uint32_t *>(ws),
                       reinterpret_cast<uint32_t *>(ws + kCbHead));
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}
