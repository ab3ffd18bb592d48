// Device half of the library: decode tables, output-index scans and the
// decode kernels for AMD Instinct MI355X (gfx950, wave64, 160 KiB LDS/CU).
//
// Hot path (gap mode): one kernel launch; per wavefront of 64 lanes, one lane
// per subsequence:
//   1. copy the tile's 32-bit units into LDS with coalesced loads;
//   2. start at k*S + gap[k] (Sec. III-C) and count the codewords that start
//      inside the subsequence (the paper's "redundant decoding" to learn
//      where each thread writes, Sec. IV-C; the chunk offsets are stored in
//      the stream, so this pass only spans one subsequence), keeping the
//      table entries it reads in registers (pair format);
//   3. wavefront exclusive scan of the counts gives each lane its output
//      index inside the tile (Sec. III-B, step 3);
//   4. write the symbols into an LDS staging tile (Sec. IV-B, Algorithm 1)
//      from the kept entries, or by decoding again, and write the tile to
//      HBM with 16-byte coalesced stores; a tile larger than the staging
//      area is written in several passes, each lane resuming where it
//      stopped.
// The decode table (first level + per-length canonical limits) lives in LDS
// for the whole persistent workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <new>
#include <vector>

#include "hd.h"
#include "hd_internal.h"

using namespace hd;

// ------------------------------------------------------------------------
// Runtime helpers
// ------------------------------------------------------------------------

namespace {

struct DeviceInfo {
    int cus = 0;
    size_t lds_per_block = 0;
    size_t lds_per_cu = 0;
    bool ok = false;
};

std::mutex g_dev_mu;
DeviceInfo g_dev[64];

const DeviceInfo *device_info()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceInfo &d = g_dev[dev];
    if (!d.ok) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess)
            return nullptr;
        d.cus = p.multiProcessorCount;
        d.lds_per_block = p.sharedMemPerBlock;
        d.lds_per_cu = p.maxSharedMemoryPerMultiProcessor ? p.maxSharedMemoryPerMultiProcessor
                                                         : p.sharedMemPerBlock;
        d.ok = true;
    }
    return &d;
}

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

// ------------------------------------------------------------------------
// Decode table
// ------------------------------------------------------------------------
//
// Device image (one allocation):
//   lut   uint32[2^k1]   indexed by the next k1 stream bits.  Single format:
//                        entry = symbol | length << 24 for codewords of at
//                        most k1 bits (symbols below 2^24); length kLenLong for a prefix of a
//                        longer codeword, kLenBad for a prefix of no
//                        codeword (for both, the symbol field holds the
//                        length the per-length search starts at: the
//                        shortest codeword under that prefix).
//                        Pair format (alphabet <= 4096, k1 <= 12):
//                        entry = sym1 | (len1 + len2) << 12 | sym2 << 16 |
//                        len2 << 28, the first codeword and, when it also
//                        fits in the k1 bits, the one after it (len2 = 0:
//                        none).  The bits a group covers, whether it holds
//                        two codewords, and both symbols as two uint16
//                        halves (entry & 0x0fff0fff) each take one step;
//                        len1 + len2 = 0 sends the lookup to the per-length
//                        limits, starting at the length in bits 0-5;
//   lim   uint64[33]     lim[l] = first canonical code of length l + number
//                        of codes of length l: a window whose l-bit prefix is
//                        below lim[l] (and whose shorter prefixes are not
//                        below theirs) holds a codeword of length l;
//   base  int64[33]      base[l] = index of the first length-l symbol in
//                        `syms` minus the first code of length l;
//   syms  uint32[n_used] used symbols sorted by (length, symbol).

struct hd_table {
    void *image = nullptr;
    uint32_t k1 = 0, L = 0, A = 0, n_used = 0;
    bool pair = false;          // first level holds up to two codewords per entry
    size_t lut_off = 0, lim_off = 0, base_off = 0, syms_off = 0, bytes = 0;
    int device = 0;
};

namespace {

constexpr uint32_t kDefaultLutBits = 12;      // pair-format tables
// Alphabets above 4096 (one-symbol entries): on the 2^18-symbol field of
// 12.6-bit mean codes 12 bits measured best (kernel 0.542 / 0.479 / 0.532 /
// 0.498 ms at 11 / 12 / 13 / 14 bits).
constexpr uint32_t kDefaultLutBitsWide = 12;

struct TableView {
    const uint32_t *lut;
    const uint64_t *lim;
    const int64_t *base;
    const uint32_t *syms;
    uint32_t k1, L;
};

inline TableView view_of(const hd_table *t)
{
    const char *p = static_cast<const char *>(t->image);
    return TableView{reinterpret_cast<const uint32_t *>(p + t->lut_off),
                     reinterpret_cast<const uint64_t *>(p + t->lim_off),
                     reinterpret_cast<const int64_t *>(p + t->base_off),
                     reinterpret_cast<const uint32_t *>(p + t->syms_off), t->k1, t->L};
}

__host__ __device__ __forceinline__ uint32_t table_lds_bytes(uint32_t k1)
{
    return (((4u << k1) + 33 * 8 + 33 * 8) + 15u) & ~15u;
}

}  // namespace

extern "C" hd_status hd_table_create(const uint8_t *lengths, const uint32_t *codes, uint32_t A,
                                     uint32_t L, uint32_t lut_bits, void *hip_stream,
                                     hd_table **out)
{
    if (!lengths || !codes || !out || A == 0 || A > HD_MAX_ALPHABET || L == 0 || L > 32)
        return HD_ERR_ARG;
    if (lut_bits != 0 && (lut_bits < 6 || lut_bits > 14))
        return HD_ERR_ARG;
    *out = nullptr;
    try {
        std::vector<uint32_t> canon(A);
        hd_status st = hd_canonical_codes_internal(lengths, A, L, canon.data());
        if (st != HD_OK)
            return st;
        uint32_t n_used = 0;
        for (uint32_t s = 0; s < A; ++s) {
            if (lengths[s] && canon[s] != codes[s])
                return HD_ERR_UNSUPPORTED;
            n_used += lengths[s] != 0;
        }
        uint32_t k1 = lut_bits ? lut_bits : (A <= 4096 ? kDefaultLutBits : kDefaultLutBitsWide);
        k1 = std::min(k1, L);
        const bool pair = A <= 4096 && k1 <= 12;

        uint64_t bl[33] = {0};
        for (uint32_t s = 0; s < A; ++s)
            bl[lengths[s]]++;
        bl[0] = 0;
        uint64_t first[34] = {0}, offs[34] = {0};
        uint64_t c = 0, o = 0;
        for (uint32_t l = 1; l <= 32; ++l) {
            c = (c + bl[l - 1]) << 1;
            first[l] = c;
            offs[l] = o;
            o += bl[l];
        }
        std::vector<uint32_t> syms(std::max<uint32_t>(n_used, 1), 0);
        {
            uint64_t fill[34];
            std::memcpy(fill, offs, sizeof(fill));
            for (uint32_t s = 0; s < A; ++s)
                if (lengths[s])
                    syms[fill[lengths[s]]++] = s;
        }
        const uint32_t nlut = 1u << k1;
        std::vector<uint32_t> lut(nlut, (kLenBad << 24) | (k1 + 1));
        // a prefix of longer codewords: the search over lengths starts at
        // the shortest codeword under it (every shorter length fails its
        // limit test for a canonical code)
        for (uint32_t s = 0; s < A; ++s) {
            const uint32_t l = lengths[s];
            if (l > k1) {
                uint32_t &e = lut[codes[s] >> (l - k1)];
                const uint32_t cur = (e >> 24) == kLenLong ? (e & 0x3fu) : 64u;
                e = (kLenLong << 24) | std::min(cur, l);
            }
        }
        for (uint32_t s = 0; s < A; ++s) {
            const uint32_t l = lengths[s];
            if (l == 0 || l > k1)
                continue;
            const uint32_t lo = codes[s] << (k1 - l), hi = (codes[s] + 1) << (k1 - l);
            for (uint32_t w = lo; w < hi; ++w)
                lut[w] = s | (l << 24);
        }
        if (pair) {
            std::vector<uint32_t> two(nlut, 0);
            for (uint32_t w = 0; w < nlut; ++w) {
                const uint32_t e = lut[w], l1 = e >> 24;
                if (l1 == kLenLong || l1 == kLenBad) {
                    two[w] = e & 0x3fu;                  // len1 + len2 = 0: per-length limits
                    continue;
                }
                uint32_t v = (e & 0xfffu) | (l1 << 12);
                if (l1 < k1) {
                    const uint32_t e2 = lut[(w << l1) & (nlut - 1)], l2 = e2 >> 24;
                    if (l2 != kLenLong && l2 != kLenBad && l2 <= k1 - l1)
                        v = (e & 0xfffu) | ((l1 + l2) << 12) | ((e2 & 0xfffu) << 16) | (l2 << 28);
                }
                two[w] = v;
            }
            lut.swap(two);
        }
        std::vector<uint64_t> lim(33, 0);
        std::vector<int64_t> base(33, 0);
        for (uint32_t l = 1; l <= 32; ++l) {
            if (l <= L) {
                lim[l] = first[l] + bl[l];
                base[l] = static_cast<int64_t>(offs[l]) - static_cast<int64_t>(first[l]);
            }
        }

        hd_table *t = new hd_table();
        t->k1 = k1;
        t->L = L;
        t->A = A;
        t->n_used = n_used;
        t->pair = pair;
        t->lut_off = 0;
        t->lim_off = align_up(size_t(4) * nlut, 16);
        t->base_off = t->lim_off + 33 * 8;
        t->syms_off = align_up(t->base_off + 33 * 8, 16);
        t->bytes = align_up(t->syms_off + 4 * syms.size(), 256);
        if (hipGetDevice(&t->device) != hipSuccess) {
            delete t;
            return HD_ERR_DEVICE;
        }
        std::vector<unsigned char> img(t->bytes, 0);
        std::memcpy(img.data() + t->lut_off, lut.data(), 4 * nlut);
        std::memcpy(img.data() + t->lim_off, lim.data(), 33 * 8);
        std::memcpy(img.data() + t->base_off, base.data(), 33 * 8);
        std::memcpy(img.data() + t->syms_off, syms.data(), 4 * syms.size());
        if (hipMalloc(&t->image, t->bytes) != hipSuccess) {
            delete t;
            return HD_ERR_NOMEM;
        }
        hipStream_t stream = static_cast<hipStream_t>(hip_stream);
        // The host image is pageable: hipMemcpyAsync from pageable memory
        // returns once the data is staged, so `img` may be freed afterwards.
        if (hipMemcpyAsync(t->image, img.data(), t->bytes, hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            (void)hipFree(t->image);
            delete t;
            return HD_ERR_DEVICE;
        }
        *out = t;
        return HD_OK;
    } catch (const std::bad_alloc &) {
        return HD_ERR_NOMEM;
    }
}

extern "C" void hd_table_destroy(hd_table *t)
{
    if (!t)
        return;
    if (t->image) {
        (void)hipDeviceSynchronize();     // no decode may still read the table
        (void)hipFree(t->image);
    }
    delete t;
}

extern "C" size_t hd_table_lds_bytes(const hd_table *t)
{
    return t ? table_lds_bytes(t->k1) : 0;
}

// ------------------------------------------------------------------------
// Device primitives
// ------------------------------------------------------------------------

namespace {

constexpr int kWave = 64;

// Inclusive prefix sum over the 64 lanes of a wavefront, in registers (DPP):
// a Kogge-Stone scan inside each row of 16 lanes (shifts 1, 2, 4, 8; a lane
// whose source lies before its row adds 0), then the row totals -- lane 15's
// into row 1 and lane 47's into row 3, then lane 31's into rows 2 and 3.
// Every lane of the wavefront must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int)
{
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false));
    return v;
}

// The wavefront's index in its workgroup, as a wavefront-uniform (scalar)
// value, so that tile and stream arithmetic derived from it stays scalar.
__device__ __forceinline__ int wave_index()
{
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

// Lane l's value, the same in every lane.
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int l)
{
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
}

__device__ __forceinline__ uint64_t lane_value64(uint64_t v, int l)
{
    return uint64_t(lane_value(static_cast<uint32_t>(v), l)) |
           (uint64_t(lane_value(static_cast<uint32_t>(v >> 32), l)) << 32);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1)
        v += __shfl_xor(v, d, kWave);
    return v;
}

// Orders this wavefront's LDS writes before its later LDS reads by other
// lanes (LDS traffic of one wavefront is processed in order; this keeps the
// compiler from moving accesses across the point).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 32 stream bits of one lane from the wavefront's transposed copy TT of its
// units: unit w of lane l sits at TT[w * 64 + l], with w = 0 a don't-care
// row (never stored, see tt_of), w = 1 .. S/32 the lane's own subsequence and
// w = S/32 + 1 the first unit of the next subsequence.  For a bit r of the subsequence, q = r + 31
// selects the unit pair (q >> 5, q >> 5 + 1) -- one ds_read2st64, all 64
// lanes on distinct banks -- and the right shift (-r) mod 32 = (~q) mod 32.
__device__ __forceinline__ uint32_t window_at(const uint32_t *TTl, uint32_t q)
{
    const uint32_t *p = TTl + (__builtin_amdgcn_ubfe(q, 5, 27) << 6);
    return __builtin_amdgcn_alignbit(p[0], p[64], ~q);
}

// Codewords longer than the first level: canonical per-length limits,
// searched from length l0 (from the slow first-level entry; at least k1 + 1),
// STEP lengths at a time.  Under a canonical code a window under the limit
// of length l is under the limit of every longer length, so the shortest
// length whose limit the window is under is the codeword's.  A step of
// several lengths issues their limit reads together: fewer dependent LDS
// round trips for latency-bound walks, more reads and registers per step.
template <int STEP = 1>
__device__ __forceinline__ uint32_t decode_long(uint32_t v, uint32_t l0, uint32_t k1, uint32_t L,
                                             const uint64_t *lim, const int64_t *base,
                                             const uint32_t *syms, uint32_t *len_out)
{
    if constexpr (STEP == 1) {
        for (uint32_t l = max(l0, k1 + 1); l <= L; ++l) {
            const uint64_t c = static_cast<uint64_t>(v) >> (32 - l);
            if (c < lim[l]) {
                *len_out = l;
                return syms[static_cast<int64_t>(c) + base[l]];
            }
        }
        *len_out = 0;
        return 0;
    }
    for (uint32_t l = max(l0, k1 + 1); l <= L; l += STEP) {
        uint32_t hit = 0;
#pragma unroll
        for (int j = STEP - 1; j >= 0; --j) {
            const uint32_t lj = min(l + j, L);
            if ((static_cast<uint64_t>(v) >> (32 - lj)) < lim[lj])
                hit = lj;
        }
        if (hit) {
            *len_out = hit;
            return syms[static_cast<int64_t>(v >> (32 - hit)) + base[hit]];
        }
    }
    *len_out = 0;
    return 0;
}

struct SmemTable {
    uint32_t *lut;
    uint64_t *lim;
    int64_t *base;
};

__device__ __forceinline__ SmemTable carve_table(unsigned char *smem, uint32_t k1)
{
    SmemTable t;
    t.lut = reinterpret_cast<uint32_t *>(smem);
    t.lim = reinterpret_cast<uint64_t *>(smem + (size_t(4) << k1));
    t.base = reinterpret_cast<int64_t *>(smem + (size_t(4) << k1) + 33 * 8);
    return t;
}

__device__ __forceinline__ void load_table(const SmemTable &t, const TableView &g)
{
    const uint32_t nlut = 1u << g.k1;
    const uint4 *src = reinterpret_cast<const uint4 *>(g.lut);
    uint4 *dst = reinterpret_cast<uint4 *>(t.lut);
    for (uint32_t i = threadIdx.x; i < nlut / 4; i += blockDim.x)
        dst[i] = src[i];
    for (uint32_t i = threadIdx.x; i < (nlut & 3u); i += blockDim.x)
        t.lut[(nlut & ~3u) + i] = g.lut[(nlut & ~3u) + i];
    if (threadIdx.x < 33) {
        t.lim[threadIdx.x] = g.lim[threadIdx.x];
        t.base[threadIdx.x] = g.base[threadIdx.x];
    }
}

// First-level lookup at relative position q - 31: up to two codewords.  A
// codeword longer than the first level (or a window matching no codeword)
// goes through the per-length limits; an invalid window reports kErrBadCode
// and consumes one bit so every loop still ends.  In the pair format a valid
// entry has len1 >= 1, so a zero group length alone flags the slow case.
template <bool PAIR>
__device__ __forceinline__ void lookup(const uint32_t *TTl, uint32_t q, const SmemTable &st,
                                       const TableView &g, uint32_t sh, uint32_t &s1,
                                       uint32_t &s2, uint32_t &l1, uint32_t &l2, uint32_t &err)
{
    const uint32_t v = window_at(TTl, q);
    const uint32_t e = st.lut[v >> sh];
    bool slow;
    if (PAIR) {
        s1 = e & 0xfffu;
        s2 = (e >> 16) & 0xfffu;
        l2 = e >> 28;
        l1 = ((e >> 12) & 0xfu) - l2;
        slow = l1 + l2 == 0;
    } else {
        s1 = e & 0xffffffu;
        s2 = 0;
        l1 = e >> 24;
        l2 = 0;
        slow = l1 - 1u >= g.k1;
    }
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(slow) != 0, 0)) {
        if (slow) {
            s1 = decode_long(v, e & 0x3fu, g.k1, g.L, st.lim, st.base, g.syms, &l1);
            l2 = 0;
            if (l1 == 0) {
                err |= kErrBadCode;
                l1 = 1;
            }
        }
    }
}

// Length a and count n of the codewords a first-level entry covers (one, or
// up to two in pair format); false for a slow entry (first codeword longer
// than k1, or no codeword at all).
template <bool PAIR>
__device__ __forceinline__ bool entry_group(uint32_t e, uint32_t k1, uint32_t &a, uint32_t &n)
{
    if (PAIR) {
        a = (e >> 12) & 0xfu;
        n = 1 + (e >= (1u << 28));
        return a != 0;
    }
    a = e >> 24;
    n = 1;
    return a - 1u < k1;
}

// Slow first group of a window (first-level entry e): one codeword through
// the per-length limits.
template <int STEP = 1>
__device__ __forceinline__ uint32_t slow_group(uint32_t v, uint32_t e, const SmemTable &st, const TableView &g,
                                               uint32_t &a, uint32_t &n, uint32_t &err)
{
    uint32_t l;
    const uint32_t s = decode_long<STEP>(v, e & 0x3fu, g.k1, g.L, st.lim, st.base, g.syms, &l);
    if (l == 0) {
        err |= kErrBadCode;
        l = 1;
    }
    a = l;
    n = 1;
    return s;
}

// Walks from q (bit position + 31) over every codeword that starts before
// qe and returns their count; q is left on the first start at or after qe.
// Two table lookups per window read: after a fast group (<= k1 <= 14 bits)
// the 32-bit window still holds at least k1 unread bits.  The loop takes
// whole groups without looking at qe (one or two codewords each, two groups
// per iteration); only the last iteration can run past qe, by at most three
// codewords (a group's second codeword, the second group, its second
// codeword), and one correction after the loop drops those that start at or
// after qe and moves q back to the first of them.
template <bool PAIR, int STEP = 1>
__device__ __forceinline__ uint32_t count_walk(const uint32_t *TTl, uint32_t &q, uint32_t qe,
                                               const SmemTable &st, const TableView &g, uint32_t sh,
                                               uint32_t &err)
{
    const uint32_t k1 = g.k1;
    uint32_t cnt = 0;
    // a1, a2: bits of the last iteration's two groups (a2 = 0: second not
    // taken); l2, m2: their second codewords' lengths (0: none); m1: the
    // second group's first length
    uint32_t a1 = 0, l2 = 0, a2 = 0, m1 = 0, m2 = 0;
    while (q < qe) {
        const uint32_t v = window_at(TTl, q);
        const uint32_t e1 = st.lut[v >> sh];
        bool fast1;
        if (PAIR) {
            a1 = (e1 >> 12) & 0xfu;
            l2 = e1 >> 28;
            fast1 = a1 != 0;
        } else {
            a1 = e1 >> 24;
            l2 = 0;
            fast1 = a1 - 1u < k1;
        }
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(!fast1) != 0, 0)) {
            if (!fast1) {
                uint32_t a, n;
                slow_group<STEP>(v, e1, st, g, a, n, err);
                a1 = a;
                l2 = 0;
            }
        }
        const uint32_t e2 = st.lut[(v << (a1 & 31u)) >> sh];
        bool fast2;
        uint32_t b2;
        if (PAIR) {
            b2 = (e2 >> 12) & 0xfu;
            m2 = e2 >> 28;
            fast2 = b2 != 0;
        } else {
            b2 = e2 >> 24;
            m2 = 0;
            fast2 = b2 - 1u < k1;
        }
        const bool take2 = fast1 && fast2;
        a2 = take2 ? b2 : 0u;
        m1 = b2 - m2;
        q += a1 + a2;
        cnt += (PAIR ? 1u + (l2 != 0) : 1u) + (take2 ? (PAIR ? 1u + (m2 != 0) : 1u) : 0u);
    }
    if (cnt != 0) {
        // starts of the last iteration's codewords after its first one
        const uint32_t q0 = q - a1 - a2;
        const uint32_t s1 = q0 + a1 - l2, s2 = q0 + a1, s3 = s2 + m1;
        const bool o1 = PAIR && l2 != 0 && s1 >= qe;
        const bool o2 = a2 != 0 && s2 >= qe;
        const bool o3 = PAIR && a2 != 0 && m2 != 0 && s3 >= qe;
        cnt -= static_cast<uint32_t>(o1) + static_cast<uint32_t>(o2) + static_cast<uint32_t>(o3);
        q = o1 ? s1 : o2 ? s2 : o3 ? s3 : q;
    }
    return cnt;
}

// Count walk that also keeps, in registers, the first-level entries of its
// first CAP iterations (pair format only): lg[2i] is iteration i's first
// group (a codeword longer than k1 becomes a one-symbol entry with a nonzero
// group-length field), lg[2i+1] its second group or 0 when that was not
// taken.  The decode step then replays the entries instead of walking the
// bits again.  nlog = iterations logged; q_cap, cnt_cap = position and count
// after them (a lane with q_cap < qe went on past the log).  Same results as
// count_walk.
template <int CAP>
__device__ __forceinline__ uint32_t count_walk_log(const uint32_t *TTl, uint32_t &q, uint32_t qe,
                                                   const SmemTable &st, const TableView &g, uint32_t sh,
                                                   uint32_t &err, uint32_t (&lg)[2 * CAP], uint32_t &nlog,
                                                   uint32_t &q_cap, uint32_t &cnt_cap)
{
    uint32_t cnt = 0;
    uint32_t a1 = 0, l2 = 0, a2 = 0, m1 = 0, m2 = 0;
    // one iteration: two groups from one window read
    auto step = [&](uint32_t &r1, uint32_t &r2) {
        const uint32_t v = window_at(TTl, q);
        uint32_t e1 = st.lut[v >> sh];
        a1 = (e1 >> 12) & 0xfu;
        l2 = e1 >> 28;
        const bool fast1 = a1 != 0;
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(!fast1) != 0, 0)) {
            if (!fast1) {
                uint32_t a, n;
                e1 = slow_group(v, e1, st, g, a, n, err) | (1u << 12);
                a1 = a;
                l2 = 0;
            }
        }
        const uint32_t e2 = st.lut[(v << (a1 & 31u)) >> sh];
        const uint32_t b2 = (e2 >> 12) & 0xfu;
        m2 = e2 >> 28;
        const bool take2 = fast1 && b2 != 0;
        a2 = take2 ? b2 : 0u;
        m1 = b2 - m2;
        q += a1 + a2;
        cnt += 1u + (l2 != 0) + (take2 ? 1u + (m2 != 0) : 0u);
        r1 = e1;
        r2 = take2 ? e2 : 0u;
    };
    nlog = 0;
    // fully unrolled: every log entry is assigned once, outside the per-lane
    // branch (a lane that has stopped logs zeros), so the log maps to fixed
    // registers
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
        uint32_t r1 = 0, r2 = 0;
        if (__builtin_amdgcn_ballot_w64(q < qe) != 0) {
            if (q < qe) {
                step(r1, r2);
                nlog = i + 1;
            }
        }
        lg[2 * i] = r1;
        lg[2 * i + 1] = r2;
    }
    q_cap = q;
    cnt_cap = cnt;
    while (q < qe) {
        uint32_t r1, r2;
        step(r1, r2);
    }
    if (cnt != 0) {
        const uint32_t q0 = q - a1 - a2;
        const uint32_t s1 = q0 + a1 - l2, s2 = q0 + a1, s3 = s2 + m1;
        const bool o1 = l2 != 0 && s1 >= qe;
        const bool o2 = a2 != 0 && s2 >= qe;
        const bool o3 = a2 != 0 && m2 != 0 && s3 >= qe;
        cnt -= static_cast<uint32_t>(o1) + static_cast<uint32_t>(o2) + static_cast<uint32_t>(o3);
        q = o1 ? s1 : o2 ? s2 : o3 ? s3 : q;
    }
    return cnt;
}

// Writes the symbols of the logged entries to dst[0 .. cnt) (the lane's whole
// output in this pass).  Steps run in lockstep over the entry index, so the
// log stays in registers; a store that would fall at or past cnt (the unused
// half of a one-codeword group, codewords of the last iteration past the
// subsequence end) goes to the lane's dummy slot.
template <int CAP, typename T>
__device__ __forceinline__ void replay_log(const uint32_t (&lg)[2 * CAP], uint32_t nlog, T *dst,
                                           uint32_t cnt, T *dummy)
{
    // A checked store picks between two base addresses (the slot's and one
    // below the dummy) and keeps its own offset, so the check costs a compare
    // and a select.
    T *const dm1 = dummy - 1;
    const uint32_t cm1 = cnt - 1;                 // cnt >= 1 whenever nlog >= 1
    uint32_t j = 0;
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
        if (static_cast<uint32_t>(i) < nlog) {
            const uint32_t e1 = lg[2 * i], e2 = lg[2 * i + 1];
            T *p = dst + j;
            p[0] = static_cast<T>(e1 & 0xfffu);   // an iteration's first codeword is always the lane's
            (j < cm1 ? p : dm1)[1] = static_cast<T>((e1 >> 16) & 0xfffu);
            j += 1u + (e1 >= (1u << 28));
            p = dst + j;
            (j < cnt ? p : dm1 + 1)[0] = static_cast<T>(e2 & 0xfffu);
            (j < cm1 ? p : dm1)[1] = static_cast<T>((e2 >> 16) & 0xfffu);
            j += (e2 != 0 ? 1u : 0u) + (e2 >= (1u << 28));
        }
    }
}

// ------------------------------------------------------------------------
// Output-index scan over chunks (Sec. III-B, step 3)
// ------------------------------------------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 8;
constexpr int kScanBlock = kScanThreads * kScanPerThread;

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *sh)
{
    v = wave_sum_u64(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        sh[w] = v;
    __syncthreads();
    uint64_t r = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i)
        r += sh[i];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *__restrict__ cc,
                                                              uint64_t M, uint64_t *partial)
{
    __shared__ uint64_t sh[kScanThreads / 64];
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kScanBlock;
    uint64_t s = 0;
    for (int i = 0; i < kScanPerThread; ++i) {
        const uint64_t c = b0 + static_cast<uint64_t>(i) * kScanThreads + threadIdx.x;
        if (c < M)
            s += cc[c];
    }
    s = block_sum_u64(s, sh);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = s;
}

// off[c] = sum of cc[0..c) for c in [0, M]; flags kErrTotal when off[M] != n.
__global__ __launch_bounds__(kScanThreads) void k_scan_finish(const uint32_t *__restrict__ cc,
                                                              uint64_t M,
                                                              const uint64_t *__restrict__ partial,
                                                              uint64_t *off, uint64_t n,
                                                              uint32_t *status)
{
    __shared__ uint64_t sh[kScanThreads / 64];
    __shared__ uint64_t tsum[kScanThreads];
    uint64_t pre = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += blockDim.x)
        pre += partial[i];
    pre = block_sum_u64(pre, sh);

    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kScanBlock;
    const uint64_t my0 = b0 + static_cast<uint64_t>(threadIdx.x) * kScanPerThread;
    uint32_t v[kScanPerThread];
    uint64_t s = 0;
    for (int i = 0; i < kScanPerThread; ++i) {
        v[i] = (my0 + i < M) ? cc[my0 + i] : 0u;
        s += v[i];
    }
    tsum[threadIdx.x] = s;
    __syncthreads();
    // exclusive scan of the 256 thread sums (Hillis-Steele in shared memory)
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const uint64_t o = threadIdx.x >= (unsigned)d ? tsum[threadIdx.x - d] : 0;
        __syncthreads();
        tsum[threadIdx.x] += o;
        __syncthreads();
    }
    uint64_t run = pre + tsum[threadIdx.x] - s;
    for (int i = 0; i < kScanPerThread; ++i) {
        if (my0 + i < M)
            off[my0 + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
        const uint64_t total = pre + tsum[kScanThreads - 1];
        off[M] = total;
        if (total != n)
            atomicOr(status, kErrTotal);
    }
}

// ------------------------------------------------------------------------
// Gap-mode decode (persistent, one lane per subsequence)
// ------------------------------------------------------------------------

constexpr uint32_t kMaxUnitsPerLane = 16;   // subsequences of at most 512 bits
// Units per lane the tile-input registers are sized for: 4 covers
// subsequences of up to 128 bits with 12 fewer registers than 16.
constexpr uint32_t kSmallUnits = 4;
// Units per lane of the middle tier: subsequences of up to 256 bits.
constexpr uint32_t kMidUnits = 8;

// One stream as the decode kernels see it.
struct StreamDev {
    const uint32_t *words;
    const uint8_t *gap;
    const uint64_t *chunk_off;   // [M + 1] output index of each chunk
    void *out;                   // n symbols of the kernel's output type
    uint64_t n, B, K, M, n_words;
    uint32_t S, stage;           // stage: staging symbols per wave (multiple of 64)
    uint32_t Cl;                 // log2 of the chunk size C (C divides 64)
    uint32_t last_bits;          // bits of the last subsequence, B - (K - 1) S
};

// log2 of a chunk size that divides 64 (checked before any launch)
inline uint32_t chunk_log2(uint32_t C)
{
    uint32_t l = 0;
    while ((2u << l) <= C)
        ++l;
    return l;
}

// Status of a decode launch: the workspace header (word 0: status bits of
// the phases before the decode kernel; word 1: the number of slots) and one
// slot per wavefront, each written once per launch (no clearing needed, so a
// gap-mode decode is a single launch).
struct GapArgs {
    StreamDev sd;
    uint32_t *head;
    uint32_t *slots;
    uint32_t own_head;           // gap mode: the kernel also writes head[0] and checks the offsets
    uint32_t *direct;            // instead of head/slots: a caller-zeroed word (pinned host memory)
                                 // that receives a wavefront's nonzero error bits by a plain store
    uint32_t direct_atomic;      // direct is device memory: OR the bits in atomically instead
    const uint32_t *list;        // when set: decode only tiles list[0 .. n_list) (one class of Alg. 2)
    uint64_t n_list;
    TableView tab;
};

// OR of err over the wavefront's lanes (every lane active).
__device__ __forceinline__ uint32_t wave_or(uint32_t e)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        e |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(e), d, kWave));
    return e;
}

// LDS of one wave's private area: the transposed unit copy TT (S/32 + 2
// words per lane, 64 lanes), the staging tile, and 64 dummy uint16 slots
// that absorb untaken second-symbol stores.
__host__ __device__ __forceinline__ uint32_t wave_units_bytes(uint32_t S)
{
    return ((S >> 5) + 1) * 64 * 4;
}

// The wavefront's TT pointer for lane `lane`: row w of TT at byte
// 256 * (w - 1) of the wavefront's area.  Row 0 is never stored: the window
// reads it only at a zero shift, where its value drops out, and it lies on
// LDS that precedes the area (the table, or the previous wavefront's area).
__device__ __forceinline__ uint32_t *tt_of(unsigned char *area, int lane)
{
    return reinterpret_cast<uint32_t *>(area) - 64 + lane;
}

// Lanes of a tile the entry probe of the self-sync kernel follows at most.
constexpr uint32_t kProbeLanes = 4;

// A sync-kernel wavefront's LDS: the transposed units, then the first
// kProbeLanes lanes' units of the tile being probed (the probe's inputs).
__host__ __device__ __forceinline__ uint32_t sync_wave_bytes(uint32_t S)
{
    return wave_units_bytes(S) + 4 * kProbeLanes * ((S >> 5) + 1);
}

__host__ __device__ __forceinline__ uint32_t wave_area_bytes(uint32_t S, uint32_t stage, uint32_t sym_bytes = 2)
{
    return wave_units_bytes(S) + sym_bytes * (stage + 64);
}

// A lane's inputs for one tile: its subsequence's units and the next unit,
// its gap byte and its successor's, and the output offsets bounding its
// chunk.  Loaded into registers (one tile ahead in the single-stream kernel).
template <uint32_t MAXU>
struct TileInT {
    uint32_t pw[MAXU];
    uint32_t pwn = 0, gk = 0, gn = 0;
    uint64_t c_lo = 0, c_hi = 0;

    // The units at src (a subsequence k < K) and the next subsequence's first
    // unit ((k+1)*S/32 < n_words for k < K).
    __device__ __forceinline__ void load_words(const uint32_t *src, uint32_t wps)
    {
        if ((wps & 3) == 0) {
#pragma unroll
            for (uint32_t i = 0; i < MAXU / 4; ++i)
                if (4 * i < wps) {
                    const uint4 v = *reinterpret_cast<const uint4 *>(src + 4 * i);
                    pw[4 * i] = v.x;
                    pw[4 * i + 1] = v.y;
                    pw[4 * i + 2] = v.z;
                    pw[4 * i + 3] = v.w;
                }
        } else {
#pragma unroll
            for (uint32_t i = 0; i < MAXU; ++i)
                if (i < wps)
                    pw[i] = src[i];
        }
        pwn = src[wps];
    }

    // Tile t (wavefront-uniform): the tile's bases are scalar, each lane adds
    // 32-bit offsets (k = 64 t + lane).
    __device__ __forceinline__ void load(const StreamDev &sd, uint64_t t, uint64_t ntiles, int lane)
    {
        if (t < ntiles) {
            const uint32_t wps = sd.S >> 5;
            const uint64_t k0 = t << 6;
            const uint64_t left = sd.K - k0;                      // subsequences from k0 on
            const uint32_t l = static_cast<uint32_t>(lane);
            if (l < left) {
                load_words(sd.words + k0 * wps + l * wps, wps);
                const uint8_t *gb = sd.gap + k0;
                gk = gb[l];
                gn = l + 1 < left ? gb[l + 1] : 0u;
                const uint64_t *cb = sd.chunk_off + (k0 >> sd.Cl);   // C divides 64
                c_lo = cb[l >> sd.Cl];                  // bounds of this lane's chunk
                c_hi = cb[(l >> sd.Cl) + 1];            // (k / C + 1 <= M for k < K)
            }
        }
    }

    __device__ __forceinline__ void store_units(uint32_t *TTl, uint32_t wps, bool act) const
    {
        if (act) {
#pragma unroll
            for (uint32_t i = 0; i < MAXU; ++i)
                if (i < wps)
                    TTl[(i + 1) * 64] = pw[i];
            TTl[(wps + 1) * 64] = pwn;
        }
    }
};

// Symbols of type T in one 16-byte group.
template <typename T>
constexpr uint32_t kGroup = 16 / sizeof(T);

// Writes staged output [g0, g1) (global indices; the stage starts at the
// 16-byte group holding g0): whole 16-byte groups with one 16-byte store per
// lane, then the partial groups at both ends (at most G - 1 symbols each, G
// = symbols per group) with one symbol store per lane on lanes 0 .. 2G-1, so
// no lane walks a group symbol by symbol.  Offsets are relative to that first
// group (32-bit).
template <typename T>
__device__ __forceinline__ void flush_stage(const StreamDev &sd, const T *stage, int lane, uint64_t g0,
                                            uint64_t g1, uint32_t &err)
{
    constexpr uint32_t G = kGroup<T>;
    if (g1 > sd.n) {
        err |= kErrOutRange;
        g1 = sd.n;
    }
    if (g0 < g1) {
        const uint64_t gb0 = g0 & ~uint64_t(G - 1);
        T *const out = static_cast<T *>(sd.out) + gb0;
        const uint32_t h0 = static_cast<uint32_t>(g0 - gb0);      // first symbol, 0..G-1
        const uint32_t e1 = static_cast<uint32_t>(g1 - gb0);      // end
        const uint32_t f0 = (h0 + G - 1) & ~(G - 1);              // first whole group
        const uint32_t f1 = e1 & ~(G - 1);                        // end of whole groups
        for (uint32_t o = f0 + G * lane; o < f1; o += G * 64)
            *reinterpret_cast<uint4 *>(out + o) = *reinterpret_cast<const uint4 *>(stage + o);
        // head [h0, min(f0, e1)) on lanes 0..G-1, tail [max(f1, f0), e1) on lanes G..2G-1
        const uint32_t ul = static_cast<uint32_t>(lane);
        const uint32_t o = ul < G ? h0 + ul : max(f1, f0) + (ul - G);
        const uint32_t lim = ul < G ? min(f0, e1) : e1;
        if (ul < 2 * G && o < lim)
            out[o] = stage[o];
    }
}

// Decodes this lane's symbols j .. jmax-1 into dst[j .. jmax), walking from q
// (the bit position of symbol j, + 31); q and j advance.  Two lookups per
// window read while at least two full groups remain; untaken slots are
// rewritten by later symbols of the lane.  The loop walks the LDS pointer
// itself.  A group's two symbols go out as two 16-bit stores: the compiler
// would merge them into one 32-bit store at a 2-byte-aligned LDS address,
// which measured far slower (the scheduling barrier keeps them apart).
template <bool PAIR, typename T>
__device__ __forceinline__ void walk_symbols(const uint32_t *TTl, uint32_t &q, uint32_t &j, uint32_t jmax,
                                             T *dst, T *dummy, const SmemTable &st,
                                             const TableView &g, uint32_t sh, uint32_t &err)
{
    const uint32_t k1 = g.k1;
    constexpr uint32_t kFastMin = PAIR ? 4u : 2u;
    if (j + kFastMin <= jmax) {
        T *pd = dst + j;
        const T *const pend = dst + (jmax - kFastMin);
        do {
            const uint32_t v = window_at(TTl, q);
            const uint32_t e1 = st.lut[v >> sh];
            uint32_t a1, n1, a2, n2;
            const bool fast1 = entry_group<PAIR>(e1, k1, a1, n1);
            uint32_t w1 = PAIR ? (e1 & 0x0fff0fffu) : (e1 & 0xffffffu);
            if (__builtin_expect(__builtin_amdgcn_ballot_w64(!fast1) != 0, 0)) {
                if (!fast1)
                    w1 = slow_group(v, e1, st, g, a1, n1, err);
            }
            // (a pair entry holds its second symbol in the upper half)
            pd[0] = static_cast<T>(PAIR ? (w1 & 0xffffu) : w1);
            __builtin_amdgcn_sched_barrier(0);
            if (PAIR)
                pd[1] = static_cast<T>(w1 >> 16);
            pd += n1;
            const uint32_t e2 = st.lut[(v << (a1 & 31u)) >> sh];
            const bool take2 = entry_group<PAIR>(e2, k1, a2, n2) && fast1;
            if (PAIR) {
                const uint32_t w2 = e2 & 0x0fff0fffu;
                pd[0] = static_cast<T>(w2 & 0xffffu);
                __builtin_amdgcn_sched_barrier(0);
                pd[1] = static_cast<T>(w2 >> 16);
            } else {
                *pd = static_cast<T>(e2 & 0xffffffu);
            }
            pd += take2 ? n2 : 0u;
            q += a1 + (take2 ? a2 : 0u);
        } while (pd <= pend);
        j = static_cast<uint32_t>(pd - dst);
    }
    while (j < jmax) {
        uint32_t s1, s2, l1, l2;
        lookup<PAIR>(TTl, q, st, g, sh, s1, s2, l1, l2, err);
        dst[j] = static_cast<T>(s1);
        ++j;
        if (PAIR) {
            // second codeword: stored when it is this lane's and in this
            // pass, else written to the lane's dummy slot
            const bool two = l2 != 0 && j < jmax;
            *(two ? dst + j : dummy) = static_cast<T>(s2);
            j += two;
            l1 += two ? l2 : 0u;
        }
        q += l1;
    }
}

// Steps 2-4 for one wavefront tile whose units are already in TT.  With
// CAP > 0 (pair format) the count step logs its table entries and a tile whose
// output fits one staging pass is decoded by replaying them.
template <bool PAIR, int CAP, typename T>
__device__ __forceinline__ void decode_tile(const StreamDev &sd, uint64_t t, int lane, uint32_t gk_in,
                                            uint32_t gn, uint64_t c_lo, uint64_t c_hi, const uint32_t *TTl,
                                            T *stage, T *dummy, const SmemTable &st,
                                            const TableView &g, uint32_t sh, uint32_t &err)
{
    static_assert(CAP == 0 || PAIR, "the entry log holds pair-format entries");
    constexpr uint32_t G = kGroup<T>;
    const uint32_t S = sd.S;
    const uint32_t PB = sd.stage - G;
    const uint64_t k0 = t << 6;                       // wavefront-uniform
    const uint64_t left = sd.K - k0;                  // subsequences from k0 on (>= 1)
    const uint32_t l = static_cast<uint32_t>(lane);
    const bool act = l < left;
    const bool last = l + 1 == left;                  // the stream's last subsequence
    const uint32_t gk = act ? gk_in : 0u;

    // 2. count pass (positions relative to the lane's subsequence start)
    const uint32_t re = act ? (last ? sd.last_bits : S) : 0u;
    uint32_t rs = gk;
    // a gap byte past any codeword, or a first subsequence not starting on
    // the stream's first bit
    if (gk >= 32 || (t == 0 && l == 0 && gk != 0)) {
        err |= kErrGapRange;
        rs = gk >= 32 ? re : rs;
    }
    if (rs > re)
        rs = re;
    const uint32_t qe = re + 31;
    uint32_t q = rs + 31;
    uint32_t lg[CAP > 0 ? 2 * CAP : 1];
    uint32_t nlog = 0, q_cap = 0, cnt_cap = 0;
    uint32_t cnt;
    if constexpr (CAP > 0)
        cnt = count_walk_log<CAP>(TTl, q, qe, st, g, sh, err, lg, nlog, q_cap, cnt_cap);
    else
        cnt = count_walk<PAIR>(TTl, q, qe, st, g, sh, err);
    // the walk must stop exactly on the next subsequence's start
    if (act) {
        const uint32_t expect = last ? re : S + gn;
        if (q - 31 != expect)
            err |= kErrLaneEnd;
    }

    // 3. output indices: wavefront scan inside the tile; the tile starts at
    //    the output offset of its first chunk (lane 0's chunk)
    const uint32_t incl = wave_incl_scan(cnt, lane);
    const uint32_t excl = incl - cnt;
    const uint32_t total = lane_value(incl, 63);
    const uint64_t gbase = lane_value64(c_lo, 0);
    {
        const uint32_t cl = lane & ((1u << sd.Cl) - 1u);
        const uint32_t excl_first = __shfl(excl, lane - cl, 64);
        if (act && (cl == (1u << sd.Cl) - 1u || last)) {
            if (gbase + excl_first != c_lo || gbase + incl != c_hi)
                err |= kErrChunkSum;
        }
    }

    // 4. decode into LDS staging, flush with 16-byte stores
    const uint32_t a0 = static_cast<uint32_t>(gbase & (G - 1));
    if constexpr (CAP > 0) {
        if (total <= PB) {
            T *dst = stage + (a0 + excl);
            replay_log<CAP>(lg, nlog, dst, cnt, dummy);
            const bool more = q_cap < qe;               // went on past the log
            if (__builtin_amdgcn_ballot_w64(more) != 0) {
                if (more) {
                    uint32_t q2 = q_cap, j2 = cnt_cap;
                    walk_symbols<PAIR>(TTl, q2, j2, cnt, dst, dummy, st, g, sh, err);
                }
            }
            wave_lds_sync();
            flush_stage(sd, stage, lane, gbase, gbase + total, err);
            wave_lds_sync();
            return;
        }
    }
    q = rs + 31;
    uint32_t j = 0;
    for (uint32_t pb = 0; pb < total; pb += PB) {
        const uint32_t lim_rel = pb + PB;
        const uint32_t jmax = lim_rel > excl ? min(cnt, lim_rel - excl) : 0u;
        // dst index of symbol j: a0 + excl + j - pb (>= a0 whenever j < jmax)
        T *dst = stage + (static_cast<int32_t>(a0 + excl) - static_cast<int32_t>(pb));
        walk_symbols<PAIR>(TTl, q, j, jmax, dst, dummy, st, g, sh, err);
        wave_lds_sync();
        flush_stage(sd, stage, lane, gbase + pb, gbase + min(lim_rel, total), err);
        wave_lds_sync();
    }
}

// Iterations whose entries the count pass logs per lane (pair format), two
// registers each.  At S <= 128 (about 22 codewords per lane at 6 bits) a
// lane needs some 6-8 iterations; a longer log costs registers and so
// occupancy, and lanes past the log finish by walking.  At S = 256 (some 30
// codewords per lane at 8 bits) the kernel holds four wavefronts per SIMD
// from 12 to 28 iterations, and a log that covers most lanes pays.
constexpr int kLogItersSmall = 8;
constexpr int kLogIters = 18;
// Entry-log length of the decode kernel for subsequences of at most
// 32 * MAXU bits.
template <uint32_t MAXU>
constexpr int log_iters()
{
    return MAXU <= kSmallUnits ? kLogItersSmall : kLogIters;
}

template <bool PAIR, uint32_t MAXU, bool LISTED = false, typename T = uint16_t>
__global__ __launch_bounds__(1024) void k_decode_gap(GapArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const TableView &g = a.tab;
    const SmemTable st = carve_table(smem, g.k1);
    load_table(st, g);
    __syncthreads();

    const StreamDev &sd = a.sd;
    const int lane = threadIdx.x & 63;
    const int wv = wave_index();
    const uint32_t wps = sd.S >> 5;
    unsigned char *area = smem + table_lds_bytes(g.k1) + wv * wave_area_bytes(sd.S, sd.stage, sizeof(T));
    uint32_t *TTl = tt_of(area, lane);
    T *stage = reinterpret_cast<T *>(area + wave_units_bytes(sd.S));
    T *dummy = stage + sd.stage + lane;
    const uint32_t sh = 32 - g.k1;

    uint32_t err = 0;
    const uint64_t ntiles = (sd.K + 63) >> 6;
    const uint32_t wpg = blockDim.x >> 6;
    const uint64_t tstride = static_cast<uint64_t>(gridDim.x) * wpg;
    // stored chunk offsets must start at 0 and end at n
    if (a.own_head && blockIdx.x == 0 && threadIdx.x == 0 && (sd.chunk_off[0] != 0 || sd.chunk_off[sd.M] != sd.n))
        err |= kErrTotal;
    // Tile inputs travel through registers one tile ahead: while tile t is
    // decoded, the inputs of the wavefront's next tile are in flight.  The
    // wavefront walks positions i, i + stride, ... of the tile sequence (all
    // tiles, or a list of them); past its end the tile index is ntiles.
    // (the list form is a separate instantiation: it costs the plain form
    // two registers, which would cut its occupancy)
    const uint64_t niter = LISTED ? a.n_list : ntiles;
    auto tile_at = [&](uint64_t j) -> uint64_t { return LISTED ? (j >= niter ? ntiles : a.list[j]) : j; };
    TileInT<MAXU> in;
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * wpg + wv;
    uint64_t t = tile_at(i);
    in.load(sd, t, ntiles, lane);
    for (; i < niter; i += tstride) {
        const bool act = (t << 6) + lane < sd.K;
        in.store_units(TTl, wps, act);
        const uint32_t gk = in.gk, gn = in.gn;
        const uint64_t c_lo = in.c_lo, c_hi = in.c_hi;
        const uint64_t tn = tile_at(i + tstride);
        in.load(sd, tn, ntiles, lane);
        wave_lds_sync();
        decode_tile<PAIR, PAIR ? log_iters<MAXU>() : 0>(sd, t, lane, gk, gn, c_lo, c_hi, TTl, stage, dummy, st, g, sh,
                                                err);
        t = tn;
    }
    err = wave_or(err);
    if (a.direct) {
        if (lane == 0 && err) {
            if (a.direct_atomic)
                atomicOr(a.direct, err);
            else
                *a.direct = err;
        }
        return;
    }
    if (lane == 0)
        a.slots[blockIdx.x * wpg + wv] = err;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.head[1] = gridDim.x * wpg;
        if (a.own_head)
            a.head[0] = 0;
    }
}

// ------------------------------------------------------------------------
// Self-synchronization (Sec. III-B-2, steps 1 and 2)
// ------------------------------------------------------------------------
//
// A tile is 64 consecutive subsequences, one per lane of a wavefront.  Every
// lane keeps a path (start, exit, count): the codewords decoded from its
// start up to its exit, the first codeword start at or after the end of its
// subsequence.  Decoding from a bit position is a deterministic walk, so two
// paths that reach one position coincide from there on; comparing positions
// is therefore an exact test of "meeting up".
//
// Step 1 (intra-tile): every lane first decodes from its raw boundary (lane
// 0 from the tile's entry).  Then, in rounds, each lane takes its
// predecessor's exit as its start.  In the first round a lane whose start
// changed simply walks its subsequence again from the new start (the raw
// path typically takes a dozen codewords to meet the true one, and a full
// walk with two lookups per window costs less than stepping both paths one
// codeword at a time that far); in later rounds it walks the new path in
// lockstep with the old one until they meet (the exit stays, the count is
// re-derived) or the new path leaves the subsequence (a new exit).
// Rounds end when a wavefront ballot finds no exit changed; after round r
// lanes 0..r agree with the entry, so at most 64 rounds are ever needed.
// The sync kernel spends at most a per-stream budget of rounds on a tile
// (sync_rounds) and lists it otherwise; the pending-tile kernel finishes
// listed tiles from per-entry exit tables (every lane walked from every
// entry g < L, then the entries chained from the tile's entry), so no
// budget ever decides the result.
//
// Step 2 (inter-tile): the entry of tile u is the exit of tile u-1's last
// lane.  Each wavefront syncs groups of consecutive tiles in order.  The
// stream's first tile, and a tile whose predecessor in its group converged
// and is exact or settled (its last exit is then final), are synced from
// their true entry and are exact.  Any other tile (the first of a group, or
// one after a tile left unconverged or unsettled) is synced from entry 0 and
// probed: the tile's first lanes are walked from every entry g < L, lane after lane,
// until all entries leave a lane j at the same exit (at most kProbeLanes
// lanes); then only lanes 0..j depend on the true entry (their starts and
// summed count per entry are recorded) and the tile's later paths and last
// exit do not (the tile is settled).  The link kernel fixes lanes 0..j of
// every settled tile whose predecessor's exit is final, and re-syncs, in
// order, runs of tiles whose entries did not converge within the probe
// (codes that never resynchronize end up here).

constexpr uint32_t kSyncRecBytes = 168;
// Tiles a sync-kernel wavefront takes at a time, in order: the first is
// probed, the others follow from their predecessors' exits.
constexpr uint64_t kChainTiles = 2;
// SyncRec::dep of an exact tile (synced from its true entry).
constexpr uint8_t kDepExact = 255;

struct SyncRec {
    uint8_t last_entry;       // next tile's lane-0 start implied by this tile's paths
    uint8_t dep;              // settled: lanes 0 .. dep-1 depend on the entry; 0: unsettled; kDepExact: exact
    uint8_t entry_used;       // the lane-0 start the tile was synced from
    uint8_t pad[5];
    uint16_t count_at[32];    // codewords of lanes 0 .. dep-1 from entry g
    uint8_t start_at[kProbeLanes - 1][32];   // start of lane i + 1 (< dep) from entry g
};
static_assert(sizeof(SyncRec) == kSyncRecBytes, "record layout");

struct SyncArgs {
    const uint32_t *words;
    uint8_t *gap_s;           // [K] sync point of every subsequence (relative)
    uint32_t *tot;            // [ntiles] codewords per tile
    SyncRec *rec;             // [ntiles]
    uint32_t *status;         // the workspace header word 0 (cleared with n_pending)
    uint32_t *n_pending;      // tiles step 1 left unconverged (zero at launch)
    uint32_t *pending;        // [ntiles] their indices
    TableView tab;
    uint64_t B, K, ntiles, n_words;
    uint32_t S;
    uint32_t rounds;          // rounds the sync kernel spends on a tile before listing it
};

// Path from relative bit r: codewords starting before E, and the first start
// at or after E (exit).
template <bool PAIR, int STEP = 1>
__device__ __forceinline__ void run_path(const uint32_t *TTc, uint32_t r, uint32_t E, const SmemTable &st,
                                         const TableView &g, uint32_t sh, uint32_t &exit, uint32_t &cnt)
{
    uint32_t q = r + 31, e = 0;
    cnt = count_walk<PAIR, STEP>(TTc, q, E + 31, st, g, sh, e);
    exit = q - 31;
}

// New path from `in` against the old path (st0, ex0, cn0): advance whichever
// position is behind, one codeword at a time, until they meet or the new one
// reaches E.  (Two-codeword steps from pair entries were measured slower here:
// these walks are short and the extra selects outweigh the saved lookups.)
template <bool PAIR>
__device__ __forceinline__ void walk_merge(const uint32_t *TTc, uint32_t in, uint32_t st0, uint32_t ex0,
                                           uint32_t cn0, uint32_t E, const SmemTable &st,
                                           const TableView &g, uint32_t sh, uint32_t &ex, uint32_t &cn)
{
    uint32_t a = in, b = st0, na = 0, nb = 0;
    for (;;) {
        if (a == b) {
            ex = ex0;
            cn = a >= E ? na : na + cn0 - nb;
            return;
        }
        if (a >= E) {
            ex = a;
            cn = na;
            return;
        }
        uint32_t s1, s2, l1, l2, e = 0;
        lookup<PAIR>(TTc, min(a, b) + 31, st, g, sh, s1, s2, l1, l2, e);
        if (a < b) {
            a += l1;
            ++na;
        } else {
            b += l1;
            ++nb;
        }
    }
}

// Loads the tile's units into the lane columns of TT (see window_at).
__device__ __forceinline__ void load_units(uint32_t *TTl, const uint32_t *words, uint64_t k, uint64_t K,
                                           uint32_t wps)
{
    if (k < K) {
        const uint32_t *src = words + k * wps;
        for (uint32_t w = 0; w < wps; ++w)
            TTl[(w + 1) * 64] = src[w];
        TTl[(wps + 1) * 64] = src[wps];
    }
}

// Step 1 for one tile with lane 0 starting at e0.
// Rounds of step 1: enough for any tile (after round r lanes 0..r are final).
constexpr uint32_t kMaxRounds = 65;
// Returns whether the rounds converged within max_rounds.
template <bool PAIR>
__device__ bool sync_tile(const uint32_t *TTl, int lane, bool act, uint32_t E, uint32_t S, uint32_t e0,
                          uint32_t max_rounds, const SmemTable &st, const TableView &g, uint32_t sh,
                          uint32_t &start, uint32_t &exit, uint32_t &cnt)
{
    start = lane == 0 ? e0 : 0u;
    exit = start;
    cnt = 0;
    if (act)
        run_path<PAIR>(TTl, start, E, st, g, sh, exit, cnt);
    for (uint32_t round = 0; round < max_rounds; ++round) {
        uint32_t in = __shfl_up(exit, 1, 64) - S;
        if (lane == 0)
            in = e0;
        bool changed = false;
        if (act && in != start) {
            uint32_t ex, cn;
            if (round == 0)
                run_path<PAIR>(TTl, in, E, st, g, sh, ex, cn);
            else
                walk_merge<PAIR>(TTl, in, start, exit, cnt, E, st, g, sh, ex, cn);
            changed = ex != exit;
            start = in;
            exit = ex;
            cnt = cn;
        }
        if (__builtin_amdgcn_ballot_w64(changed) == 0)
            return true;
    }
    return false;
}

// Per-lane subsequence end: S, or the stream end for the last subsequence.
__device__ __forceinline__ uint32_t lane_end(uint64_t k, uint64_t K, uint64_t B, uint32_t S)
{
    if (k >= K)
        return 0;
    return k + 1 == K ? static_cast<uint32_t>(B - k * S) : S;
}

// The tile's totals after step 1 (wavefront-uniform).
struct TileSync {
    uint32_t total, last_exit;    // codewords of the tile; its last lane's exit
    bool done;                    // the rounds converged
    bool off_end;                 // the stream's last subsequence (in this tile) ends off the stream end
};

// Runs step 1 on tile t (lane 0 starting at e0), stores the sync points and,
// when the rounds do not converge within max_rounds, lists the tile.
template <bool PAIR>
__device__ TileSync sync_core(const SyncArgs &a, uint64_t t, const uint32_t *TTl, int lane, uint32_t e0,
                              uint32_t max_rounds, const SmemTable &st, const TableView &g, uint32_t sh)
{
    const uint32_t S = a.S;
    const uint64_t k = (t << 6) + lane;
    const bool act = k < a.K;
    const uint32_t E = lane_end(k, a.K, a.B, S);
    uint32_t start, exit, cnt;
    const bool done = sync_tile<PAIR>(TTl, lane, act, E, S, e0, max_rounds, st, g, sh, start, exit, cnt);
    // the stream's last subsequence must end exactly on the stream end (a
    // codeword path that runs past it found no consistent sync point)
    const bool off_end = k + 1 == a.K && exit != E;
    // only the round-limited pass lists tiles (each at most once, so the
    // list index stays below ntiles); kMaxRounds always converges
    if (!done && max_rounds < kMaxRounds && lane == 0)
        a.pending[atomicAdd(a.n_pending, 1u)] = static_cast<uint32_t>(t);
    if (act)
        a.gap_s[k] = static_cast<uint8_t>(start);
    TileSync r;
    r.total = static_cast<uint32_t>(wave_sum_u64(cnt));
    r.last_exit = __shfl(exit, 63, 64);
    r.done = done;
    r.off_end = __builtin_amdgcn_ballot_w64(off_end) != 0;
    return r;
}

// Re-syncs tile t from its true entry e0 with enough rounds (the link step)
// and stores its total; returns the next tile's entry.
template <bool PAIR>
__device__ uint32_t resync_tile(const SyncArgs &a, uint64_t t, const uint32_t *TTl, int lane, uint32_t e0,
                                const SmemTable &st, const TableView &g, uint32_t sh)
{
    const TileSync r = sync_core<PAIR>(a, t, TTl, lane, e0, kMaxRounds, st, g, sh);
    if (lane == 0) {
        if (r.off_end)
            atomicOr(a.status, kErrNoSync);
        a.tot[t] = r.total;
        a.rec[t].last_entry = static_cast<uint8_t>(r.last_exit - a.S);
    }
    return r.last_exit - a.S;
}

// The entry probe of a tile synced from entry 0: lanes 0..31 follow the
// tile from entries 0..31 (entries from L on are not followed).  Each walks
// the tile's lane-0 subsequence from its entry and, while the entries leave
// lane i's subsequence at different exits, lane i + 1's subsequence from its
// own exit, up to lane kProbeLanes - 1.  When all entries leave lane j at one
// exit, every later path of the tile is independent of the entry: returns
// j + 1 and records the summed count of lanes 0..j and the starts of lanes
// 1..j per entry (for the link step); 0 when no common exit is found within
// the probe or the stream ends first.  cols holds the probe lanes' units
// (word w of lane i at cols[(w - 1) * kProbeLanes + i]); every lane copies
// the column it walks into its own TT column first, so the walks read
// conflict-free.
template <bool PAIR>
__device__ uint32_t probe_tile(const SyncArgs &a, uint64_t t, uint32_t *TTl, const uint32_t *cols, int lane,
                               const SmemTable &st, const TableView &g, uint32_t sh)
{
    const uint32_t S = a.S, wps = S >> 5;
    const uint32_t gent = static_cast<uint32_t>(lane);
    const bool probe = gent < 32 && gent < g.L;
    SyncRec *rec = a.rec + t;
    uint32_t cur = gent, sum = 0, dep = 0;
    wave_lds_sync();
    for (uint32_t i = 0; i < kProbeLanes; ++i) {
        const uint64_t k = (t << 6) + i;
        if (k >= a.K)
            break;                                   // the stream ends first: unsettled
        for (uint32_t w = 1; w <= wps + 1; ++w)
            TTl[w * 64] = cols[(w - 1) * kProbeLanes + i];
        uint32_t ex = 0, c = 0;
        if (probe)
            run_path<PAIR>(TTl, cur, lane_end(k, a.K, a.B, S), st, g, sh, ex, c);
        const uint32_t ref = __shfl(ex, 0, 64);
        sum += c;
        cur = ex - S;
        if (__builtin_amdgcn_ballot_w64(probe && ex != ref) == 0) {
            dep = i + 1;
            break;
        }
        if (probe && i + 1 < kProbeLanes)
            rec->start_at[i][gent] = static_cast<uint8_t>(cur);
    }
    if (gent < 32)
        rec->count_at[gent] = static_cast<uint16_t>(probe ? sum : 0u);
    return dep;
}

// Copies the first kProbeLanes lanes' units of the tile in TT (c0 = lane 0's
// column) to cols in the probe's layout.
__device__ __forceinline__ void save_probe_cols(uint32_t *cols, const uint32_t *c0, uint32_t ul, uint32_t wps)
{
    for (uint32_t f = ul; f < (wps + 1) * kProbeLanes; f += 64)
        cols[f] = c0[(f / kProbeLanes + 1) * 64 + f % kProbeLanes];
}

template <int WPG, bool PAIR>
__global__ __launch_bounds__(WPG * 64) __attribute__((amdgpu_waves_per_eu(8))) void k_ss_sync(SyncArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const TableView &g = a.tab;
    const SmemTable st = carve_table(smem, g.k1);
    load_table(st, g);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = wave_index();
    const uint32_t wps = a.S >> 5;
    unsigned char *area = smem + table_lds_bytes(g.k1) + wv * sync_wave_bytes(a.S);
    uint32_t *TTl = tt_of(area, lane);
    // the probe lanes' units of the tile being probed (the probe's layout)
    uint32_t *cols = reinterpret_cast<uint32_t *>(area + wave_units_bytes(a.S));
    const uint32_t *c0 = TTl - lane;                   // lane 0's column
    const uint32_t sh = 32 - g.k1;
    // groups of kChainTiles consecutive tiles, dealt to the wavefronts in
    // turn (slow regions of a stream spread over many wavefronts)
    const uint64_t ngroups = (a.ntiles + kChainTiles - 1) / kChainTiles;
    const uint64_t gstride = static_cast<uint64_t>(gridDim.x) * WPG;
    for (uint64_t gi = static_cast<uint64_t>(blockIdx.x) * WPG + wv; gi < ngroups; gi += gstride) {
        const uint64_t t_begin = gi * kChainTiles;
        const uint64_t t_end = min(a.ntiles, t_begin + kChainTiles);
        // the entry of the next tile, when final (the stream's first tile starts
        // at entry 0)
        bool chained = t_begin == 0;
        uint32_t entry = 0;
        for (uint64_t t = t_begin; t < t_end; ++t) {
            load_units(TTl, a.words, (t << 6) + lane, a.K, wps);
            wave_lds_sync();
            const uint32_t e0 = chained ? entry : 0u;
            const TileSync r = sync_core<PAIR>(a, t, TTl, lane, e0, a.rounds, st, g, sh);
            uint32_t dep = kDepExact;
            if (!chained) {
                save_probe_cols(cols, c0, static_cast<uint32_t>(lane), wps);
                dep = probe_tile<PAIR>(a, t, TTl, cols, lane, st, g, sh);
            }
            if (lane == 0) {
                SyncRec *rec = a.rec + t;
                rec->last_entry = static_cast<uint8_t>(r.last_exit - a.S);
                rec->dep = static_cast<uint8_t>(dep);
                rec->entry_used = static_cast<uint8_t>(e0);
                a.tot[t] = r.total;
                // the tile's paths are final when its entry is, or does not
                // matter past the probed lanes, and the rounds converged;
                // otherwise a later kernel decides
                if (r.off_end && r.done && dep != 0)
                    atomicOr(a.status, kErrNoSync);
            }
            chained = r.done && dep != 0;
            entry = r.last_exit - a.S;
            wave_lds_sync();
        }
    }
}

// Finishes step 1 for the tiles the sync kernel left unconverged after
// its round budget (listed in a.pending; typically streams that do not
// self-synchronize, such as long runs of one codeword, where rounds would
// fix one lane at a time).  One workgroup per tile: its wavefronts walk
// every lane's subsequence from every entry g < L (exit and count per entry,
// in LDS), then the lane entries are chained through those tables from the
// entry the tile was synced from (0, or its predecessor's exit for a
// chained tile); the tile's probe record, if any, is already written.
// LDS: table, the tile's units (one copy), exit and count tables.
// While every workgroup has at most one listed tile (few), the walks are
// latency-bound (a handful of tiles, typically of long codewords): the
// workgroup's 16 wavefronts share one tile's entries and search the
// per-length limits four lengths per step.  With more tiles they are
// throughput-bound: each half of the workgroup (8 wavefronts) takes its own
// tile, one length per step.
constexpr int kPendingWaves = 16;
constexpr int kPendingStep = 4;

// LDS of one tile in the pending-tile kernel: its units (one copy), exit
// and count tables, lane entries and the blocked chain's maps.
__host__ __device__ __forceinline__ uint32_t pending_tile_bytes(uint32_t S)
{
    return (wave_units_bytes(S) + 64 * 32 * 3 + 64 + 8 * 32 + 8 + 15u) & ~15u;
}

template <bool PAIR>
__global__ __launch_bounds__(kPendingWaves * 64) __attribute__((amdgpu_waves_per_eu(8))) void k_ss_pending(SyncArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const uint32_t n = *a.n_pending;
    const bool few = n <= gridDim.x;
    const uint32_t per = few ? 1u : 2u;          // tiles per workgroup pass
    if (blockIdx.x * per >= n)
        return;                                  // no listed tile for this workgroup
    const TableView &g = a.tab;
    const SmemTable st = carve_table(smem, g.k1);
    load_table(st, g);
    const int lane = threadIdx.x & 63;
    const uint32_t wv = static_cast<uint32_t>(wave_index());
    const uint32_t half = few ? 0u : wv / (kPendingWaves / 2);
    const uint32_t hw = few ? wv : wv % (kPendingWaves / 2);          // wavefront within the half
    const uint32_t hwaves = few ? kPendingWaves : kPendingWaves / 2;
    const uint32_t htid = threadIdx.x - half * (kPendingWaves / 2) * 64;
    const uint32_t wps = a.S >> 5;
    unsigned char *units = smem + table_lds_bytes(g.k1) + half * pending_tile_bytes(a.S);
    const uint32_t *TTl = tt_of(units, lane);
    uint8_t *exo = units + wave_units_bytes(a.S);                       // [64][32] exit - E
    uint16_t *cnt = reinterpret_cast<uint16_t *>(exo + 64 * 32);        // [64][32]
    uint8_t *ent = reinterpret_cast<uint8_t *>(cnt + 64 * 32);          // [64] entry of each lane
    uint8_t *bmap = ent + 64;                                           // [8][32] exit of 8 lanes per entry
    uint8_t *bent = bmap + 8 * 32;                                      // [8] entry of each block of 8 lanes
    const uint32_t sh = 32 - g.k1;
    const uint32_t ne = min(g.L, 32u);
    // every thread runs every pass and barrier; a half without a tile in the
    // last pass only waits
    for (uint32_t pass = blockIdx.x; pass * per < n; pass += gridDim.x) {
        const uint32_t i = pass * per + half;
        const bool have = i < n;
        const uint64_t t = have ? a.pending[i] : 0u;
        const uint64_t k = (t << 6) + lane;
        const bool act = have && k < a.K;
        __syncthreads();                     // the previous tiles are done with the LDS
        if (hw == 0 && have)
            load_units(tt_of(units, lane), a.words, k, a.K, wps);
        __syncthreads();
        const uint32_t E = lane_end(k, a.K, a.B, a.S);
        if (have) {
            for (uint32_t e = hw; e < ne; e += hwaves) {
                uint32_t ex = e, c = 0;
                if (act) {
                    if (few)
                        run_path<PAIR, kPendingStep>(TTl, e, E, st, g, sh, ex, c);
                    else
                        run_path<PAIR, 1>(TTl, e, E, st, g, sh, ex, c);
                }
                exo[lane * 32 + e] = static_cast<uint8_t>(ex - E);
                cnt[lane * 32 + e] = static_cast<uint16_t>(c);
            }
        }
        __syncthreads();
        // Chain the lane entries from the tile's entry in three steps of
        // eight dependent reads: each block of eight lanes maps every entry
        // to the block's exit, one thread chains the eight blocks, then each
        // block walks its lanes from its own entry.
        if (have && htid < 256 && (htid & 31u) < ne) {
            const uint32_t b = htid >> 5;
            uint32_t e = htid & 31u;
            for (uint32_t l = 8 * b; l < 8 * b + 8; ++l)
                if ((t << 6) + l < a.K)
                    e = exo[l * 32 + e];
            bmap[htid] = static_cast<uint8_t>(e);
        }
        __syncthreads();
        if (have && htid == 0) {
            uint32_t e = a.rec[t].entry_used;
            for (uint32_t b = 0; b < 8; ++b) {
                bent[b] = static_cast<uint8_t>(e);
                e = bmap[b * 32 + e];
            }
            a.rec[t].last_entry = static_cast<uint8_t>(e);
            // the stream's last tile, final when its entry is (tile 0) or
            // does not matter: its last path must end on the stream end
            // (e is that lane's exit minus its end)
            if ((t + 1) << 6 >= a.K && (t == 0 || a.rec[t].dep != 0) && e != 0)
                atomicOr(a.status, kErrNoSync);
        }
        __syncthreads();
        if (have && htid < 8) {
            uint32_t e = bent[htid];
            for (uint32_t l = 8 * htid; l < 8 * htid + 8; ++l) {
                ent[l] = static_cast<uint8_t>(e);
                if ((t << 6) + l < a.K)
                    e = exo[l * 32 + e];
            }
        }
        __syncthreads();
        if (have && hw == 0) {
            const uint32_t e = ent[lane];
            const uint32_t c = act ? cnt[lane * 32 + e] : 0u;
            if (act)
                a.gap_s[k] = static_cast<uint8_t>(e);
            const uint32_t total = static_cast<uint32_t>(wave_sum_u64(c));
            if (lane == 0)
                a.tot[t] = total;
        }
    }
}

// LDS of the pending-tile kernel: the table and two tiles.
__host__ __device__ __forceinline__ uint32_t pending_lds_bytes(uint32_t k1, uint32_t S)
{
    return table_lds_bytes(k1) + 2 * pending_tile_bytes(S);
}

// Clears the pending-tile count and the status header word before the
// synchronization kernels run (a kernel, not a memset, so the sequence can be
// captured in a graph).
__global__ void k_ss_clear(uint32_t *n_pending, uint32_t *status)
{
    if (threadIdx.x == 0) {
        *n_pending = 0;
        *status = 0;
    }
}

// Step 2's link: one lane per tile fixes the entry-dependent lanes of every
// settled tile whose predecessor's last exit is final; each run of unsettled
// tiles from a final entry is re-synced in order by the wavefront that holds
// its first tile.
template <int WPG, bool PAIR>
__global__ __launch_bounds__(WPG * 64) void k_ss_link(SyncArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const TableView &g = a.tab;
    const SmemTable st = carve_table(smem, g.k1);
    load_table(st, g);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = wave_index();
    const uint32_t wps = a.S >> 5;
    uint32_t *TTl = tt_of(smem + table_lds_bytes(g.k1) + wv * wave_units_bytes(a.S), lane);
    const uint32_t sh = 32 - g.k1;
    // One lane per tile, 64 consecutive tiles per wavefront pass, so the
    // record reads of all of them are in flight together.
    for (uint64_t base = (static_cast<uint64_t>(blockIdx.x) * WPG + wv) << 6; base < a.ntiles;
         base += static_cast<uint64_t>(gridDim.x) * WPG * 64) {
        const uint64_t u = base + lane;
        // tile 0 starts at the true stream start; a tile whose probe found a
        // common exit has a last exit that does not depend on its entry
        bool head = false;
        uint32_t e = 0, dep = 0;
        if (u >= 1 && u < a.ntiles && (u == 1 || a.rec[u - 1].dep != 0)) {
            head = true;
            e = a.rec[u - 1].last_entry;
            dep = a.rec[u].dep;
        }
        if (head && dep != 0 && dep != kDepExact) {
            // lanes 0 .. dep-1 under the true entry e
            const SyncRec *r = a.rec + u;
            a.gap_s[u << 6] = static_cast<uint8_t>(e);
            for (uint32_t i = 1; i < dep; ++i)
                a.gap_s[(u << 6) + i] = r->start_at[i - 1][e];
            a.tot[u] = a.tot[u] + r->count_at[e] - r->count_at[0];
        }
        // runs of tiles the probe left open, each from a final entry:
        // re-synced in order by the whole wavefront
        uint64_t runs = __builtin_amdgcn_ballot_w64(head && dep == 0);
        while (runs != 0) {
            const int l = __builtin_ctzll(runs);
            runs &= runs - 1;
            uint32_t ev = __shfl(e, l, 64);
            for (uint64_t v = base + l; v < a.ntiles; ++v) {
                // (a tile that follows an unsettled one was synced from entry
                // 0, never chained, so it is settled or unsettled here)
                const uint32_t dv = v == base + l ? 0u : a.rec[v].dep;
                if (dv != 0 && dv != kDepExact) {
                    if (lane == 0) {
                        a.gap_s[v << 6] = static_cast<uint8_t>(ev);
                        a.tot[v] = a.tot[v] + a.rec[v].count_at[ev] - a.rec[v].count_at[0];
                    } else if (static_cast<uint32_t>(lane) < dv) {
                        a.gap_s[(v << 6) + lane] = a.rec[v].start_at[lane - 1][ev];
                    }
                    break;
                }
                load_units(TTl, a.words, (v << 6) + lane, a.K, wps);
                wave_lds_sync();
                ev = resync_tile<PAIR>(a, v, TTl, lane, ev, st, g, sh);
                wave_lds_sync();
            }
        }
    }
}

// ------------------------------------------------------------------------
// The paper's Algorithm 2, literally: compression-ratio classes of tiles
// ------------------------------------------------------------------------
//
// Sec. IV-C, Alg. 2: every sequence's compression ratio (known from an
// earlier phase -- here the stored chunk offsets give each wavefront tile's
// symbol count) is classified into T_high + 1 groups, (0,1], (1,2], ...,
// (T_high - 1, T_high] and (T_high, 16]; the classes are histogrammed and
// the tile indices key-value sorted by class on the device; the histogram
// goes to the host, which prefix-sums it and launches one decode kernel per
// non-empty class, each with a staging buffer sized for its class's upper
// bound, on its own stream.  Kept as an ablation beside the persistent
// single-launch decode.

constexpr uint32_t kCrMaxClasses = 17;      // T_high <= 16, plus the class above it

struct CrArgs {
    const uint64_t *chunk_off;
    uint64_t ntiles, M, n, B;
    uint32_t S, Cl, t_high;
    uint32_t *cls;           // [ntiles] class of each tile (0-based)
    uint32_t *hist;          // [kCrMaxClasses]
    uint32_t *cursor;        // [kCrMaxClasses]
    uint32_t *order;         // [ntiles] tile indices sorted by class
    uint32_t *head;          // status header (word 0 cleared here, word 1 = 0: no slots)
};

__global__ void k_cr_clear(CrArgs a)
{
    const uint32_t i = threadIdx.x;
    if (i < kCrMaxClasses) {
        a.hist[i] = 0;
        a.cursor[i] = 0;
    }
    if (i == 0) {
        // the stored offsets must start at 0 and end at n
        a.head[0] = (a.chunk_off[0] != 0 || a.chunk_off[a.M] != a.n) ? kErrTotal : 0u;
        a.head[1] = 0;
    }
}

// ClassifyCR + ParHistogram: a tile's compression ratio is its output bits
// (16 per symbol) over its input bits; class c (1-based) holds ratios in
// (c - 1, c], the last class everything above T_high.
__global__ __launch_bounds__(256) void k_cr_classify(CrArgs a)
{
    __shared__ uint32_t h[kCrMaxClasses];
    if (threadIdx.x < kCrMaxClasses)
        h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < a.ntiles) {
        const uint64_t c0 = (t << 6) >> a.Cl, c1 = min(((t + 1) << 6) >> a.Cl, a.M);
        const uint64_t count = a.chunk_off[c1] - a.chunk_off[c0];
        const uint64_t bits = min(uint64_t(64) * a.S, a.B - (t << 6) * a.S);
        // ceil(16 count / bits), at least 1, classes above T_high merged
        const uint64_t cr = (16 * count + bits - 1) / max(bits, uint64_t(1));
        const uint32_t c = static_cast<uint32_t>(min<uint64_t>(max<uint64_t>(cr, 1), a.t_high + 1)) - 1;
        a.cls[t] = c;
        atomicAdd(&h[c], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kCrMaxClasses && h[threadIdx.x])
        atomicAdd(&a.hist[threadIdx.x], h[threadIdx.x]);
}

// ParKeyValueSort of (class, tile index) by class: a counting sort.  Each
// wavefront takes one atomic slot range per class present among its lanes
// (order within a class is not kept: it only affects scheduling).
__global__ __launch_bounds__(256) void k_cr_sort(CrArgs a)
{
    __shared__ uint32_t start[kCrMaxClasses];
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t c = 0; c < kCrMaxClasses; ++c) {
            start[c] = acc;
            acc += a.hist[c];
        }
    }
    __syncthreads();
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool act = t < a.ntiles;
    const uint32_t c = act ? a.cls[t] : kCrMaxClasses;
    uint64_t left = __builtin_amdgcn_ballot_w64(act);
    while (left) {
        const uint32_t cc = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(c), __builtin_ctzll(left)));
        const uint64_t mine = __builtin_amdgcn_ballot_w64(act && c == cc);
        const uint32_t lane = threadIdx.x & 63;
        const uint32_t rank = static_cast<uint32_t>(__builtin_popcountll(mine & ((uint64_t(1) << lane) - 1)));
        uint32_t base = 0;
        if (lane == static_cast<uint32_t>(__builtin_ctzll(mine)))
            base = atomicAdd(&a.cursor[cc], static_cast<uint32_t>(__builtin_popcountll(mine)));
        base = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(base), __builtin_ctzll(mine)));
        if (act && c == cc)
            a.order[start[cc] + base + rank] = static_cast<uint32_t>(t);
        left &= ~mine;
    }
}

// ------------------------------------------------------------------------
// Batched persistent decode: many streams, one launch
// ------------------------------------------------------------------------
//
// The paper groups sequences by compression ratio and launches one decode
// kernel per group, each with its own shared-memory size, on separate
// streams (Sec. IV-C, Alg. 2).  Here one persistent launch covers every
// stream of a batch, its LDS layout reserving the largest table, subsequence
// and staging of the batch.  A work item is WPG consecutive wavefront tiles
// of one stream (items never straddle streams); items are numbered stream by
// stream and workgroup b takes items b, b + grid, b + 2 grid, ...  The item
// sequence of a workgroup is fixed, so every wave of it knows when the next
// item belongs to another stream: only then do the waves meet at a barrier
// while the stream's table is loaded into LDS.  Otherwise waves run on their
// own, with the next item's tile inputs in registers while the current tile
// decodes, as in the single-stream kernel.  Chunk offsets are the streams'
// own (stored by the encoder); the status word comes zeroed with the
// uploaded descriptors.

struct BatchStreamDev {
    StreamDev sd;
    TableView tab;
    uint64_t item0;       // first work item of this stream (within its launch)
    uint64_t ntiles;
    uint32_t pair;
    uint32_t pad;
};

struct BatchArgs {
    const BatchStreamDev *streams;
    uint32_t n_streams;
    uint64_t n_items;
    uint32_t *status;            // device word OR-ed atomically, or (direct) a caller-zeroed word
    uint32_t direct;             // status is pinned host memory: a nonzero error is stored, not OR-ed
    uint32_t S_alloc, stage_alloc, k1_alloc;
};

// Last stream at or after `from` whose first item is <= item (empty streams
// share their successor's item0 and are stepped over).
__device__ __forceinline__ uint32_t batch_stream_of(const BatchArgs &a, uint64_t item, uint32_t from)
{
    uint32_t s = from;
    while (s + 1 < a.n_streams && a.streams[s + 1].item0 <= item)
        ++s;
    return s;
}

// Table formats a batch launch must handle: all pair, all one-symbol, or both.
constexpr int kBatchPairOnly = 0, kBatchWideOnly = 1, kBatchMixed = 2;

template <int FORMATS, uint32_t MAXU>
__global__ __launch_bounds__(1024) void k_decode_batch(BatchArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wv = wave_index();
    unsigned char *area = smem + table_lds_bytes(a.k1_alloc) + wv * wave_area_bytes(a.S_alloc, a.stage_alloc);
    uint32_t *TTl = tt_of(area, lane);
    uint16_t *stage = reinterpret_cast<uint16_t *>(area + wave_units_bytes(a.S_alloc));
    uint16_t *dummy = stage + a.stage_alloc + lane;
    uint32_t err = 0;
    const uint32_t wpg = blockDim.x >> 6;
    const uint64_t istride = gridDim.x;
    uint64_t item = blockIdx.x;
    uint32_t si = batch_stream_of(a, item, 0);
    uint32_t cur = 0xffffffffu;
    TileInT<MAXU> in;
    if (item < a.n_items) {
        const BatchStreamDev &b0 = a.streams[si];
        in.load(b0.sd, (item - b0.item0) * wpg + wv, b0.ntiles, lane);
    }
    for (; item < a.n_items; item += istride) {
        const BatchStreamDev &bs = a.streams[si];
        if (si != cur) {
            __syncthreads();                 // every wave is done with the previous table
            load_table(carve_table(smem, bs.tab.k1), bs.tab);
            __syncthreads();
            cur = si;
        }
        const uint64_t t = (item - bs.item0) * wpg + wv;
        const bool live = t < bs.ntiles;
        in.store_units(TTl, bs.sd.S >> 5, live && (t << 6) + lane < bs.sd.K);
        const uint32_t gk = in.gk, gn = in.gn;
        const uint64_t c_lo = in.c_lo, c_hi = in.c_hi;
        const uint64_t nitem = item + istride;
        const uint32_t nsi = nitem < a.n_items ? batch_stream_of(a, nitem, si) : si;
        if (nitem < a.n_items) {
            const BatchStreamDev &nb = a.streams[nsi];
            in.load(nb.sd, (nitem - nb.item0) * wpg + wv, nb.ntiles, lane);
        }
        wave_lds_sync();
        // a stream's stored offsets must start at 0 and end at its n
        if (live && t == 0 && lane == 0 &&
            (bs.sd.chunk_off[0] != 0 || bs.sd.chunk_off[bs.sd.M] != bs.sd.n))
            err |= kErrTotal;
        if (live) {
            const SmemTable st = carve_table(smem, bs.tab.k1);
            const uint32_t sh = 32 - bs.tab.k1;
            if (FORMATS == kBatchPairOnly || (FORMATS == kBatchMixed && bs.pair))
                decode_tile<true, MAXU == kSmallUnits ? kLogItersSmall : 0>(bs.sd, t, lane, gk, gn, c_lo, c_hi, TTl,
                                                                       stage, dummy, st, bs.tab, sh, err);
            else
                decode_tile<false, 0>(bs.sd, t, lane, gk, gn, c_lo, c_hi, TTl, stage, dummy, st, bs.tab, sh, err);
        }
        si = nsi;
    }
    if (err) {
        if (a.direct)
            *a.status = err;
        else
            atomicOr(a.status, err);
    }
}

}  // namespace

// ------------------------------------------------------------------------
// Host entry points
// ------------------------------------------------------------------------

namespace {

constexpr size_t kWsHeader = 256;          // status header: word 0 status bits, word 1 slot count
// Status slots after the header: one per resident wavefront of a decode
// launch (the plan keeps grid x waves per workgroup within this).
constexpr uint32_t kMaxSlots = 8192;
constexpr size_t kWsStatusBytes = kWsHeader + 4 * size_t(kMaxSlots);

constexpr uint32_t kMaxWavesPerGroup = 16;    // 1024 work-items
constexpr uint32_t kMaxWavesPerCu = 32;       // 8 wavefronts per SIMD

struct Plan {
    uint32_t wpg, stage, groups_per_cu;
    uint32_t lds_bytes;
    uint32_t grid;
};

// Raises a kernel's dynamic-LDS limit to the device's per-workgroup maximum
// (once per kernel); launches and occupancy queries both need it.
bool allow_full_lds(const void *func)
{
    static std::mutex mu;
    static std::vector<const void *> done;
    std::lock_guard<std::mutex> lk(mu);
    if (std::find(done.begin(), done.end(), func) != done.end())
        return true;
    const DeviceInfo *dev = device_info();
    if (!dev || hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(dev->lds_per_block)) != hipSuccess)
        return false;
    done.push_back(func);
    return true;
}

// Workgroups of `threads` work-items with `lds` bytes of dynamic LDS that
// the runtime reports resident per CU for a kernel (memoized); -1 when the
// query fails.
int resident_groups(const void *func, uint32_t threads, size_t lds)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, uint32_t, size_t>, int> memo;
    const auto key = std::make_tuple(func, threads, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end())
            return it->second;
    }
    int nb = -1;
    if (!allow_full_lds(func) ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, func, static_cast<int>(threads), lds) != hipSuccess)
        nb = -1;
    std::lock_guard<std::mutex> lk(mu);
    memo[key] = nb;
    return nb;
}

// Resident wavefronts per CU that a kernel's vector registers allow
// (512 per SIMD lane, allocated in blocks of 8; at most 8 per SIMD).
uint32_t reg_waves_per_cu(const void *func)
{
    static std::mutex mu;
    static std::vector<std::pair<const void *, uint32_t>> memo;
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &m : memo)
        if (m.first == func)
            return m.second;
    uint32_t waves = 32;
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, func) == hipSuccess && at.numRegs > 0) {
        const uint32_t alloc = (static_cast<uint32_t>(at.numRegs) + 7) / 8 * 8;
        waves = 4 * std::max<uint32_t>(1, std::min<uint32_t>(8, 512 / alloc));
    }
    memo.emplace_back(func, waves);
    return waves;
}

template <bool PAIR, typename T>
const void *gap_kernel_of(uint32_t S)
{
    if (S <= 32 * kSmallUnits)
        return reinterpret_cast<const void *>(&k_decode_gap<PAIR, kSmallUnits, false, T>);
    if (S <= 32 * kMidUnits)
        return reinterpret_cast<const void *>(&k_decode_gap<PAIR, kMidUnits, false, T>);
    return reinterpret_cast<const void *>(&k_decode_gap<PAIR, kMaxUnitsPerLane, false, T>);
}

// The decode kernel for a table format, subsequence size and symbol width.
const void *gap_kernel(bool pair, uint32_t S, uint32_t w = 2)
{
    if (w == 1)
        return pair ? gap_kernel_of<true, uint8_t>(S) : gap_kernel_of<false, uint8_t>(S);
    if (w == 4)
        return pair ? gap_kernel_of<true, uint32_t>(S) : gap_kernel_of<false, uint32_t>(S);
    return pair ? gap_kernel_of<true, uint16_t>(S) : gap_kernel_of<false, uint16_t>(S);
}

// Symbol width of a stream (0 reads as 2).
inline uint32_t sym_bytes(const hd_stream_info &i) { return i.symbol_bytes ? i.symbol_bytes : 2u; }

hd_status check_stream(const hd_dstream *s, hd_mode m)
{
    if (!s || !s->table)
        return HD_ERR_ARG;
    const hd_stream_info &i = s->info;
    const hd_table *t = s->table;
    if (i.subseq_bits < 32 || i.subseq_bits % 32 != 0)
        return HD_ERR_ARG;
    if (i.subseq_bits > 32 * kMaxUnitsPerLane)
        return HD_ERR_UNSUPPORTED;
    if (i.chunk_subseqs == 0)
        return HD_ERR_ARG;
    if (i.alphabet_size != t->A || i.max_len != t->L)
        return HD_ERR_ARG;
    // the alphabet must fit the symbol width
    const uint32_t w = sym_bytes(i);
    if (!((w == 1 && i.alphabet_size <= 256u) || (w == 2 && i.alphabet_size <= 65536u) ||
          (w == 4 && i.alphabet_size <= HD_MAX_ALPHABET)))
        return HD_ERR_ARG;
    const uint64_t K = ceil_div(i.n_bits, i.subseq_bits);
    if (i.n_subseq != K || i.n_chunks != ceil_div(K, i.chunk_subseqs))
        return HD_ERR_ARG;
    if (i.n_words < K * (i.subseq_bits / 32) + 2)
        return HD_ERR_ARG;
    if (i.n_bits > i.n_symbols * uint64_t(i.max_len) || i.n_bits < i.n_symbols)
        return HD_ERR_CORRUPT;
    if (K && !s->words)
        return HD_ERR_ARG;
    if (m == HD_MODE_GAP) {
        if (64 % i.chunk_subseqs != 0)
            return HD_ERR_UNSUPPORTED;
        if ((K && !s->gap) || !s->chunk_offsets)
            return HD_ERR_ARG;
    } else if (m != HD_MODE_SELF_SYNC) {
        return HD_ERR_ARG;
    }
    return HD_OK;
}

// Default staging: a wavefront tile of 64 subsequences decodes about
// 64 * S / (mean code length) symbols; a quarter of headroom keeps nearly
// every tile to one staging pass.
uint32_t auto_stage_for(const hd_stream_info &si)
{
    const double per_tile = si.n_bits ? 64.0 * si.subseq_bits * double(si.n_symbols) / double(si.n_bits) : 1024.0;
    uint32_t st = static_cast<uint32_t>(per_tile * 1.25) + 64;
    return std::min<uint32_t>(8192, std::max<uint32_t>(512, (st + 255) / 256 * 256));
}

// Wavefronts per workgroup with the most resident wavefronts per CU for a
// workgroup LDS footprint of table + wpg * area (ties: the smaller
// workgroup).  The table is shared by a workgroup's wavefronts, so larger
// workgroups amortize it.  The rule is conservative where measurement showed
// the naive one wrong: workgroups come in multiples of 4 wavefronts (spread
// evenly over the 4 SIMDs of a CU), at most 7 wavefronts per SIMD (scalar
// registers), 4 KB of a CU's LDS kept in reserve, and never more
// workgroups than the runtime reports resident.  Workgroups of 13 or 14
// wavefronts, or LDS filled to the last kilobytes, measured 30 % slower: the
// last workgroup of each CU did not become resident with the others.
constexpr uint32_t kSimdWaveCap = 7;
constexpr uint32_t kLdsReserve = 4096;

uint64_t lds_cu_usable(const DeviceInfo *dev)
{
    return dev->lds_per_cu > kLdsReserve ? dev->lds_per_cu - kLdsReserve : dev->lds_per_cu;
}

uint32_t occupancy_wpg(uint32_t table, uint32_t area, const DeviceInfo *dev, uint32_t *waves = nullptr,
                       uint32_t cap = kMaxWavesPerCu, const void *func = nullptr)
{
    cap = std::min<uint32_t>(cap, 4 * kSimdWaveCap);
    const uint64_t lds_cu = lds_cu_usable(dev);
    uint32_t best = 0, best_waves = 0;
    for (uint32_t w = 4; w <= kMaxWavesPerGroup; w += 4) {
        const uint64_t lds = table + uint64_t(w) * area;
        if (lds > dev->lds_per_block)
            break;
        uint32_t fit = std::min<uint32_t>(static_cast<uint32_t>(lds_cu / lds), cap / w);
        const int nb = func ? resident_groups(func, w * 64, lds) : -1;
        if (nb >= 0)
            fit = std::min<uint32_t>(fit, static_cast<uint32_t>(nb));
        if (fit * w > best_waves) {
            best = w;
            best_waves = fit * w;
        }
    }
    if (best == 0 && table + uint64_t(area) <= dev->lds_per_block) {
        best = 1;                      // a layout so large that only one wavefront fits
        best_waves = 1;
    }
    if (waves)
        *waves = best_waves;
    return best;
}

// Largest staging size (a multiple of 64) whose layout still keeps `target`
// wavefronts resident per CU; 256 when none does.
uint32_t stage_for_waves(uint32_t table, uint32_t S, uint32_t target, const DeviceInfo *dev)
{
    for (uint32_t st = 16384; st > 256; st -= 64) {
        uint32_t waves = 0;
        occupancy_wpg(table, wave_area_bytes(S, st), dev, &waves);
        if (waves >= target)
            return st;
    }
    return 256;
}

// Default staging of a stream: within 1.05 .. 1.25 times the mean tile
// output (+64), the size that keeps the most wavefronts resident per CU,
// the larger one among equals (tiles above it are written in passes).
uint32_t occupancy_stage(const hd_stream_info &si, uint32_t table, uint32_t reg_cap, const DeviceInfo *dev,
                         const void *func)
{
    const double per_tile = si.n_bits ? 64.0 * si.subseq_bits * double(si.n_symbols) / double(si.n_bits) : 1024.0;
    auto clamp64 = [](double v) {
        const uint32_t st = (static_cast<uint32_t>(v) + 63) / 64 * 64;
        return std::min<uint32_t>(8192, std::max<uint32_t>(512, st));
    };
    const uint32_t lo = clamp64(per_tile * 1.05 + 64), hi = clamp64(per_tile * 1.25 + 64);
    uint32_t best = hi, best_waves = 0;
    for (uint32_t st = hi; st >= lo; st -= 64) {
        uint32_t waves = 0;
        occupancy_wpg(table, wave_area_bytes(si.subseq_bits, st, sym_bytes(si)), dev, &waves, reg_cap, func);
        if (waves > best_waves) {
            best = st;
            best_waves = waves;
        }
        if (st < 64 + 512)
            break;
    }
    return best;
}

hd_status make_plan(const hd_dstream *s, const hd_tune *tune, Plan *p)
{
    const DeviceInfo *dev = device_info();
    if (!dev)
        return HD_ERR_DEVICE;
    const uint32_t S = s->info.subseq_bits;
    const void *func = gap_kernel(s->table->pair, S, sym_bytes(s->info));
    const uint32_t reg_cap = reg_waves_per_cu(func);
    const uint32_t table = table_lds_bytes(s->table->k1);
    p->stage = tune && tune->stage_symbols ? tune->stage_symbols
                                           : occupancy_stage(s->info, table, reg_cap, dev, func);
    if (p->stage < 256 || p->stage > 16384 || p->stage % 64)
        return HD_ERR_ARG;
    const uint32_t area = wave_area_bytes(S, p->stage, sym_bytes(s->info));
    p->wpg = tune && tune->waves_per_group ? tune->waves_per_group
                                           : occupancy_wpg(table, area, dev, nullptr, reg_cap, func);
    if (p->wpg == 0)
        return HD_ERR_UNSUPPORTED;                   // not even one wavefront fits
    if (p->wpg > kMaxWavesPerGroup)
        return HD_ERR_ARG;
    p->lds_bytes = table + p->wpg * area;
    if (p->lds_bytes > dev->lds_per_block)
        return HD_ERR_UNSUPPORTED;
    uint32_t fit = static_cast<uint32_t>(lds_cu_usable(dev) / p->lds_bytes);
    fit = std::max<uint32_t>(1, std::min<uint32_t>(fit, std::min<uint32_t>(reg_cap, 4 * kSimdWaveCap) / p->wpg));
    const int nb = resident_groups(func, p->wpg * 64, p->lds_bytes);
    if (nb > 0)
        fit = std::min<uint32_t>(fit, static_cast<uint32_t>(nb));
    p->groups_per_cu = tune && tune->groups_per_cu ? std::min(tune->groups_per_cu, fit) : fit;
    const uint64_t ntiles = ceil_div(s->info.n_subseq, 64);
    const uint64_t want = ceil_div(ntiles, p->wpg);
    const uint64_t cap = std::min<uint64_t>(uint64_t(dev->cus) * p->groups_per_cu, kMaxSlots / p->wpg);
    p->grid = static_cast<uint32_t>(std::max<uint64_t>(1, std::min(want, cap)));
    return HD_OK;
}

// Gap mode: the status area only (the chunk offsets are the stream's).
size_t gap_ws_bytes() { return kWsStatusBytes; }

// The status area plus an output-index scan over M chunks: offsets [M + 1]
// and the scan's block partials.
size_t scan_ws_bytes(uint64_t M)
{
    const uint64_t nblk = std::max<uint64_t>(1, ceil_div(M, kScanBlock));
    return kWsStatusBytes + align_up(8 * (M + 1), 256) + align_up(8 * nblk, 256);
}

// ------------------------------------------------------------------------
// Self-sync host side (workspace, launches of the synchronization kernels)
// ------------------------------------------------------------------------

// Self-sync workspace: the gap-mode part sized for one chunk per tile, then
// the found sync points, per-tile totals and per-tile records.
struct SyncWs {
    uint8_t *gap_s;
    uint32_t *tot;
    SyncRec *rec;
    uint32_t *n_pending;
    uint32_t *pending;
};

size_t sync_ws_bytes(uint64_t K)
{
    const uint64_t nt = ceil_div(K, 64);
    return scan_ws_bytes(nt) + align_up(K, 256) + 2 * align_up(4 * nt, 256) + align_up(kSyncRecBytes * nt, 256) +
           256;
}

SyncWs sync_ws(void *workspace, uint64_t K)
{
    const uint64_t nt = ceil_div(K, 64);
    char *p = static_cast<char *>(workspace) + scan_ws_bytes(nt);
    SyncWs w;
    w.gap_s = reinterpret_cast<uint8_t *>(p);
    p += align_up(K, 256);
    w.tot = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * nt, 256);
    w.rec = reinterpret_cast<SyncRec *>(p);
    p += align_up(kSyncRecBytes * nt, 256);
    w.pending = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * nt, 256);
    w.n_pending = reinterpret_cast<uint32_t *>(p);
    return w;
}

template <int WPG, bool PAIR>
hd_status launch_sync(const SyncArgs &a, uint32_t grid, uint32_t lds, hipStream_t stream)
{
    static bool attr_set = false;
    if (!attr_set) {
        const int lim = static_cast<int>(device_info()->lds_per_block);
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ss_sync<WPG, PAIR>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ss_link<WPG, PAIR>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ss_pending<PAIR>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
            return HD_ERR_DEVICE;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_ss_sync<WPG, PAIR>), dim3(grid), dim3(WPG * 64), lds, stream, a);
    hipLaunchKernelGGL((k_ss_pending<PAIR>), dim3(grid), dim3(kPendingWaves * 64),
                       pending_lds_bytes(a.tab.k1, a.S), stream, a);
    // the link kernel takes 64 tiles per wavefront
    const uint32_t lgrid = static_cast<uint32_t>(
        std::max<uint64_t>(1, std::min<uint64_t>(grid, ceil_div(a.ntiles, uint64_t(64) * WPG))));
    hipLaunchKernelGGL((k_ss_link<WPG, PAIR>), dim3(lgrid), dim3(WPG * 64), lds, stream, a);
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}

// Rounds the sync kernel spends on a tile before listing it for the
// pending-tile kernel (which finishes any tile exactly, so the budget only
// trades time).  Longer codes resynchronize later: a tile needs more rounds,
// and listing it costs L walks per lane.  Measured budgets (whole self-sync
// step): config 2 (mean code 5.9 bits) 2 / 3 / 4 / 6 / 8 rounds 0.333 /
// 0.336 / 0.358 / 0.394 / 0.418 ms; config 3 (7.4 bits) 3 / 4 / 6 / 8 / 12
// rounds 0.992 / 0.985 / 0.964 / 0.975 / 0.969 ms; the config-2 field as
// uint32 codes (12.6 bits) 4 / 6 / 8 / 12 / 16 rounds 7.90 / 5.30 / 4.15 /
// 3.66 / 3.64 ms.
uint32_t sync_rounds(const hd_stream_info &i)
{
    const double lbar = i.n_symbols ? double(i.n_bits) / double(i.n_symbols) : 1.0;
    return lbar < 7.0 ? 3u : lbar < 10.0 ? 6u : 16u;
}

// Enqueues steps 1-2 of self-synchronization: sync points into gap_s and
// per-tile codeword totals into tot.
hd_status enqueue_sync(const hd_dstream *s, const SyncWs &w, uint32_t *status, hipStream_t stream)
{
    const DeviceInfo *dev = device_info();
    if (!dev)
        return HD_ERR_DEVICE;
    const hd_stream_info &i = s->info;
    constexpr int kWpg = 8;
    const uint32_t lds = table_lds_bytes(s->table->k1) + kWpg * sync_wave_bytes(i.subseq_bits);
    if (lds > dev->lds_per_block)
        return HD_ERR_UNSUPPORTED;
    // four groups of eight waves per CU measured faster here than three
    const uint32_t fit = std::max<uint32_t>(1, std::min<uint32_t>(static_cast<uint32_t>(dev->lds_per_cu / lds), 32 / kWpg));
    const uint64_t nt = ceil_div(i.n_subseq, 64);
    const uint32_t grid = static_cast<uint32_t>(
        std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(ceil_div(nt, kChainTiles), kWpg), uint64_t(dev->cus) * fit)));
    SyncArgs a;
    a.words = s->words;
    a.gap_s = w.gap_s;
    a.tot = w.tot;
    a.rec = w.rec;
    a.status = status;
    a.n_pending = w.n_pending;
    a.pending = w.pending;
    a.tab = view_of(s->table);
    a.B = i.n_bits;
    a.K = i.n_subseq;
    a.ntiles = nt;
    a.n_words = i.n_words;
    a.S = i.subseq_bits;
    a.rounds = sync_rounds(i);
    return s->table->pair ? launch_sync<kWpg, true>(a, grid, lds, stream)
                          : launch_sync<kWpg, false>(a, grid, lds, stream);
}

// ------------------------------------------------------------------------
// Gap-kernel launch (both modes)
// ------------------------------------------------------------------------

template <bool PAIR, uint32_t MAXU, typename T = uint16_t>
hd_status launch_gap(const GapArgs &a, const Plan &p, hipStream_t stream)
{
    if (!allow_full_lds(reinterpret_cast<const void *>(&k_decode_gap<PAIR, MAXU, false, T>)))
        return HD_ERR_DEVICE;
    hipLaunchKernelGGL((k_decode_gap<PAIR, MAXU, false, T>), dim3(p.grid), dim3(p.wpg * 64), p.lds_bytes, stream,
                       a);
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}

template <typename T>
hd_status launch_gap_as(const GapArgs &a, const Plan &p, bool pair, uint32_t S, hipStream_t stream)
{
    if (pair)
        return S <= 32 * kSmallUnits ? launch_gap<true, kSmallUnits, T>(a, p, stream)
               : S <= 32 * kMidUnits ? launch_gap<true, kMidUnits, T>(a, p, stream)
                                     : launch_gap<true, kMaxUnitsPerLane, T>(a, p, stream);
    return S <= 32 * kSmallUnits ? launch_gap<false, kSmallUnits, T>(a, p, stream)
           : S <= 32 * kMidUnits ? launch_gap<false, kMidUnits, T>(a, p, stream)
                                 : launch_gap<false, kMaxUnitsPerLane, T>(a, p, stream);
}

// Enqueues the scan of per-tile totals (self-sync mode): off[0..M].
hd_status enqueue_chunk_scan(const uint32_t *cc, uint64_t M, uint64_t n, uint64_t *off,
                             uint64_t *partial, uint32_t *status, hipStream_t stream)
{
    const uint64_t nblk = std::max<uint64_t>(1, ceil_div(M, kScanBlock));
    if (nblk > 0x7fffffffu)
        return HD_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kScanThreads), 0, stream, cc, M, partial);
    hipLaunchKernelGGL(k_scan_finish, dim3(nblk), dim3(kScanThreads), 0, stream, cc, M, partial,
                       off, n, status);
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}

}  // namespace

extern "C" hd_status hd_decode_workspace_size(const hd_dstream *s, hd_mode m, const hd_tune *tune,
                                              size_t *bytes)
{
    (void)tune;
    if (!bytes)
        return HD_ERR_ARG;
    hd_status st = check_stream(s, m);
    if (st != HD_OK)
        return st;
    *bytes = m == HD_MODE_GAP ? gap_ws_bytes() : sync_ws_bytes(s->info.n_subseq);
    return HD_OK;
}

namespace {

struct WsView {
    uint32_t *status;    // header word 0
    uint32_t *slots;     // [kMaxSlots]
    uint64_t *off;       // [M + 1] output index of each tile (self-sync mode)
    uint64_t *partial;   // scan partials (self-sync mode)
};

WsView ws_view(void *workspace, uint64_t M)
{
    char *ws = static_cast<char *>(workspace);
    WsView v;
    v.status = reinterpret_cast<uint32_t *>(ws);
    v.slots = reinterpret_cast<uint32_t *>(ws + kWsHeader);
    v.off = reinterpret_cast<uint64_t *>(ws + kWsStatusBytes);
    v.partial = reinterpret_cast<uint64_t *>(ws + kWsStatusBytes + align_up(8 * (M + 1), 256));
    return v;
}

hd_status check_call(const hd_dstream *s, hd_mode m, const hd_tune *tune, void *workspace,
                     size_t ws_bytes)
{
    hd_status st = check_stream(s, m);
    if (st != HD_OK)
        return st;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 ||
        reinterpret_cast<uintptr_t>(s->words) % 16 != 0)
        return HD_ERR_ARG;
    size_t need = 0;
    st = hd_decode_workspace_size(s, m, tune, &need);
    if (st != HD_OK)
        return st;
    return ws_bytes < need ? HD_ERR_ARG : HD_OK;
}

}  // namespace

extern "C" hd_status hd_decode_prepare(const hd_dstream *s, hd_mode m, const hd_tune *tune,
                                       void *workspace, size_t ws_bytes, void *hip_stream)
{
    hd_status st = check_call(s, m, tune, workspace, ws_bytes);
    if (st != HD_OK)
        return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const hd_stream_info &i = s->info;
    if (m == HD_MODE_GAP)
        return HD_OK;          // the output indices are the stream's stored chunk offsets
    // self-sync: steps 1-2 find the sync points and tile totals, step 3 scans
    // the totals (one chunk per tile)
    const uint64_t nt = ceil_div(i.n_subseq, 64);
    const WsView w = ws_view(workspace, nt);
    const SyncWs sw = sync_ws(workspace, i.n_subseq);
    // the status word is cleared once, here, before any kernel of the call
    // can report into it
    hipLaunchKernelGGL(k_ss_clear, dim3(1), dim3(64), 0, stream, sw.n_pending, w.status);
    if (i.n_subseq) {
        st = enqueue_sync(s, sw, w.status, stream);
        if (st != HD_OK)
            return st;
    }
    return enqueue_chunk_scan(sw.tot, nt, i.n_symbols, w.off, w.partial, w.status, stream);
}

namespace {

// The decode-and-write launch of a checked call.  direct: a caller-zeroed
// status word (gap mode only; the workspace is then not used).
hd_status run_decode_kernel(const hd_dstream *s, void *out, hd_mode m, const hd_tune *tune, void *workspace,
                            uint32_t *direct, hipStream_t stream, bool direct_atomic = false)
{
    hd_status st = HD_OK;
    const hd_stream_info &i = s->info;
    const bool ss = m == HD_MODE_SELF_SYNC;
    const uint64_t M = ss ? ceil_div(i.n_subseq, 64) : i.n_chunks;
    // (an empty stream still launches the kernel: it writes the status)
    const WsView w = workspace ? ws_view(workspace, M) : WsView{nullptr, nullptr, nullptr, nullptr};
    Plan p;
    st = make_plan(s, tune, &p);
    if (st != HD_OK)
        return st;
    GapArgs a;
    a.sd.words = s->words;
    a.sd.gap = ss ? sync_ws(workspace, i.n_subseq).gap_s : s->gap;
    a.sd.chunk_off = ss ? w.off : s->chunk_offsets;
    a.sd.out = out;
    a.sd.n = i.n_symbols;
    a.sd.B = i.n_bits;
    a.sd.K = i.n_subseq;
    a.sd.M = M;
    a.sd.n_words = i.n_words;
    a.sd.S = i.subseq_bits;
    a.sd.last_bits = i.n_subseq ? static_cast<uint32_t>(i.n_bits - (i.n_subseq - 1) * i.subseq_bits) : 0u;
    a.sd.Cl = ss ? 6u : chunk_log2(i.chunk_subseqs);
    a.sd.stage = p.stage;
    a.head = w.status;
    a.slots = w.slots;
    a.own_head = ss ? 0u : 1u;
    a.direct = direct;
    a.direct_atomic = direct_atomic ? 1u : 0u;
    a.list = nullptr;
    a.n_list = 0;
    a.tab = view_of(s->table);
    const uint32_t wid = sym_bytes(i);
    if (wid == 1)
        return launch_gap_as<uint8_t>(a, p, s->table->pair, i.subseq_bits, stream);
    if (wid == 4)
        return launch_gap_as<uint32_t>(a, p, s->table->pair, i.subseq_bits, stream);
    return launch_gap_as<uint16_t>(a, p, s->table->pair, i.subseq_bits, stream);
}

}  // namespace

extern "C" hd_status hd_decode_run(const hd_dstream *s, void *out, hd_mode m, const hd_tune *tune,
                                   void *workspace, size_t ws_bytes, void *hip_stream)
{
    hd_status st = check_call(s, m, tune, workspace, ws_bytes);
    if (st != HD_OK)
        return st;
    if ((s->info.n_symbols && !out) || reinterpret_cast<uintptr_t>(out) % 16 != 0)
        return HD_ERR_ARG;
    return run_decode_kernel(s, out, m, tune, workspace, nullptr, static_cast<hipStream_t>(hip_stream));
}

hd_status hd::decode_gap_direct(const hd_dstream *s, uint16_t *out, uint32_t *status_word, void *hip_stream)
{
    hd_status st = check_stream(s, HD_MODE_GAP);
    if (st != HD_OK)
        return st;
    if (sym_bytes(s->info) != 2)
        return HD_ERR_UNSUPPORTED;
    if (!status_word || (s->info.n_symbols && !out) || reinterpret_cast<uintptr_t>(out) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(s->words) % 16 != 0)
        return HD_ERR_ARG;
    return run_decode_kernel(s, out, HD_MODE_GAP, nullptr, nullptr, status_word, static_cast<hipStream_t>(hip_stream));
}

extern "C" hd_status hd_decode(const hd_dstream *s, void *out, hd_mode m, const hd_tune *tune,
                               void *workspace, size_t ws_bytes, void *hip_stream)
{
    hd_status st = check_call(s, m, tune, workspace, ws_bytes);
    if (st != HD_OK)
        return st;
    if ((s->info.n_symbols && !out) || reinterpret_cast<uintptr_t>(out) % 16 != 0)
        return HD_ERR_ARG;
    st = hd_decode_prepare(s, m, tune, workspace, ws_bytes, hip_stream);
    if (st != HD_OK)
        return st;
    return hd_decode_run(s, out, m, tune, workspace, ws_bytes, hip_stream);
}

// ------------------------------------------------------------------------
// Algorithm 2 host side: classes, per-class launches on separate streams
// ------------------------------------------------------------------------

namespace {

// Library-owned streams of the per-class launches (default priority, one
// per class, created once per device) and their completion events.
struct CrStreams {
    hipStream_t s[kCrMaxClasses];
    hipEvent_t ev[kCrMaxClasses];
    bool ok = false;
};

std::mutex g_cr_mu;
CrStreams g_cr[64];

const CrStreams *cr_streams()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_cr_mu);
    CrStreams &c = g_cr[dev];
    if (!c.ok) {
        for (uint32_t i = 0; i < kCrMaxClasses; ++i)
            if (hipStreamCreateWithFlags(&c.s[i], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&c.ev[i], hipEventDisableTiming) != hipSuccess)
                return nullptr;
        c.ok = true;
    }
    return &c;
}

struct CrWs {
    uint32_t *head, *cls, *order, *hist, *cursor;
};

size_t cr_ws_bytes(uint64_t ntiles)
{
    return kWsStatusBytes + 2 * align_up(4 * ntiles, 256) + 2 * 256;
}

CrWs cr_ws(void *workspace, uint64_t ntiles)
{
    char *p = static_cast<char *>(workspace);
    CrWs w;
    w.head = reinterpret_cast<uint32_t *>(p);
    p += kWsStatusBytes;
    w.cls = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * ntiles, 256);
    w.order = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * ntiles, 256);
    w.hist = reinterpret_cast<uint32_t *>(p);
    w.cursor = reinterpret_cast<uint32_t *>(p + 256);
    return w;
}

// Staging of class c (1-based): a tile of 64 subsequences of S bits at a
// compression ratio of at most c holds at most 4 S c symbols (+ 64 for the
// alignment of the first 16-byte group).
uint32_t cr_stage(uint32_t S, uint32_t c)
{
    return std::min<uint32_t>(16384, (4 * S * c + 64 + 63) / 64 * 64);
}

template <bool PAIR, uint32_t MAXU>
hd_status launch_listed(const GapArgs &a, const Plan &p, hipStream_t stream)
{
    const void *f = reinterpret_cast<const void *>(&k_decode_gap<PAIR, MAXU, true>);
    if (!allow_full_lds(f))
        return HD_ERR_DEVICE;
    hipLaunchKernelGGL((k_decode_gap<PAIR, MAXU, true>), dim3(p.grid), dim3(p.wpg * 64), p.lds_bytes, stream, a);
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}

const void *listed_kernel(bool pair, uint32_t S)
{
    const bool small = S <= 32 * kSmallUnits;
    if (pair)
        return small ? reinterpret_cast<const void *>(&k_decode_gap<true, kSmallUnits, true>)
                     : reinterpret_cast<const void *>(&k_decode_gap<true, kMaxUnitsPerLane, true>);
    return small ? reinterpret_cast<const void *>(&k_decode_gap<false, kSmallUnits, true>)
                 : reinterpret_cast<const void *>(&k_decode_gap<false, kMaxUnitsPerLane, true>);
}

}  // namespace

extern "C" hd_status hd_decode_cr_classes_workspace_size(const hd_dstream *s, size_t *bytes)
{
    if (!bytes)
        return HD_ERR_ARG;
    hd_status st = check_stream(s, HD_MODE_GAP);
    if (st != HD_OK)
        return st;
    if (sym_bytes(s->info) != 2)
        return HD_ERR_UNSUPPORTED;
    *bytes = cr_ws_bytes(ceil_div(s->info.n_subseq, 64));
    return HD_OK;
}

extern "C" hd_status hd_decode_cr_classes(const hd_dstream *s, uint16_t *out, void *workspace, size_t ws_bytes,
                                          void *hip_stream, hd_cr_classes *report)
{
    size_t need = 0;
    hd_status st = hd_decode_cr_classes_workspace_size(s, &need);
    if (st != HD_OK)
        return st;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || ws_bytes < need ||
        reinterpret_cast<uintptr_t>(s->words) % 16 || (s->info.n_symbols && !out) ||
        reinterpret_cast<uintptr_t>(out) % 16)
        return HD_ERR_ARG;
    const hd_stream_info &i = s->info;
    const uint64_t nt = ceil_div(i.n_subseq, 64);
    if (nt > 0xffffffffu)
        return HD_ERR_UNSUPPORTED;
    const auto t_entry = std::chrono::steady_clock::now();
    const DeviceInfo *dev = device_info();
    const CrStreams *cs = cr_streams();
    if (!dev || !cs)
        return HD_ERR_DEVICE;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const uint32_t S = i.subseq_bits;
    const uint32_t table = table_lds_bytes(s->table->k1);
    const void *func = listed_kernel(s->table->pair, S);
    const uint32_t reg_cap = reg_waves_per_cu(func);
    // T_high: the largest class whose staging still leaves a quarter of the
    // wavefront slots of a CU (8 of 32) resident -- the paper's rule (25 %
    // occupancy) on this architecture
    uint32_t t_high = 1;
    for (uint32_t c = 1; c <= kCrMaxClasses - 1; ++c) {
        uint32_t waves = 0;
        occupancy_wpg(table, wave_area_bytes(S, cr_stage(S, c)), dev, &waves, reg_cap, func);
        if (waves >= kMaxWavesPerCu / 4)
            t_high = c;
    }
    const CrWs w = cr_ws(workspace, nt);
    CrArgs ca;
    ca.chunk_off = s->chunk_offsets;
    ca.ntiles = nt;
    ca.M = i.n_chunks;
    ca.n = i.n_symbols;
    ca.B = i.n_bits;
    ca.S = S;
    ca.Cl = chunk_log2(i.chunk_subseqs);
    ca.t_high = t_high;
    ca.cls = w.cls;
    ca.hist = w.hist;
    ca.cursor = w.cursor;
    ca.order = w.order;
    ca.head = w.head;
    // device: classify, histogram, key-value sort (lines 2-7 of the figure)
    hipLaunchKernelGGL(k_cr_clear, dim3(1), dim3(64), 0, stream, ca);
    const uint32_t g = static_cast<uint32_t>(std::max<uint64_t>(1, ceil_div(nt, 256)));
    if (nt) {
        hipLaunchKernelGGL(k_cr_classify, dim3(g), dim3(256), 0, stream, ca);
        hipLaunchKernelGGL(k_cr_sort, dim3(g), dim3(256), 0, stream, ca);
    }
    // host: the histogram comes back, its prefix sum gives each class's
    // first position in the sorted tile list
    uint32_t hist[kCrMaxClasses] = {0};
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hist, w.hist, sizeof(hist), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return HD_ERR_DEVICE;
    uint32_t start[kCrMaxClasses];
    uint32_t acc = 0;
    for (uint32_t c = 0; c < kCrMaxClasses; ++c) {
        start[c] = acc;
        acc += hist[c];
    }
    if (acc != nt)
        return HD_ERR_DEVICE;
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->t_high = t_high;
        report->classify_us =
            std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t_entry).count();
    }
    // one decode launch per non-empty class, each with its class's staging,
    // on its own stream; the caller's stream waits for all of them
    for (uint32_t c = 0; c <= t_high; ++c) {
        if (!hist[c])
            continue;
        hd_tune tune{0, cr_stage(S, std::min(c + 1, t_high)), 0, 0};
        Plan p;
        st = make_plan(s, &tune, &p);
        if (st != HD_OK)
            return st;
        GapArgs a;
        a.sd.words = s->words;
        a.sd.gap = s->gap;
        a.sd.chunk_off = s->chunk_offsets;
        a.sd.out = out;
        a.sd.n = i.n_symbols;
        a.sd.B = i.n_bits;
        a.sd.K = i.n_subseq;
        a.sd.M = i.n_chunks;
        a.sd.n_words = i.n_words;
        a.sd.S = S;
        a.sd.last_bits = static_cast<uint32_t>(i.n_bits - (i.n_subseq - 1) * S);
        a.sd.Cl = chunk_log2(i.chunk_subseqs);
        a.sd.stage = p.stage;
        a.head = w.head;
        a.slots = nullptr;
        a.own_head = 0;
        a.direct = w.head;
        a.direct_atomic = 1;
        a.list = w.order + start[c];
        a.n_list = hist[c];
        a.tab = view_of(s->table);
        // the plan sized the grid for every tile; this class has hist[c]
        const uint64_t want = ceil_div(hist[c], p.wpg);
        p.grid = static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(want, p.grid)));
        const bool small = S <= 32 * kSmallUnits;
        hipStream_t cst = cs->s[c];
        st = s->table->pair ? (small ? launch_listed<true, kSmallUnits>(a, p, cst)
                                     : launch_listed<true, kMaxUnitsPerLane>(a, p, cst))
                            : (small ? launch_listed<false, kSmallUnits>(a, p, cst)
                                     : launch_listed<false, kMaxUnitsPerLane>(a, p, cst));
        if (st != HD_OK)
            return st;
        if (hipEventRecord(cs->ev[c], cst) != hipSuccess || hipStreamWaitEvent(stream, cs->ev[c], 0) != hipSuccess)
            return HD_ERR_DEVICE;
        if (report) {
            report->tiles[c] = hist[c];
            report->stage_symbols[c] = p.stage;
            report->waves_per_group[c] = p.wpg;
            report->launches += 1;
        }
    }
    return HD_OK;
}

extern "C" hd_status hd_decode_sync_points(const hd_dstream *s, const void *workspace, size_t ws_bytes,
                                          uint8_t *gap_out, void *hip_stream)
{
    hd_status st = check_stream(s, HD_MODE_SELF_SYNC);
    if (st != HD_OK)
        return st;
    if (!workspace || ws_bytes < sync_ws_bytes(s->info.n_subseq) || (s->info.n_subseq && !gap_out))
        return HD_ERR_ARG;
    if (s->info.n_subseq == 0)
        return HD_OK;
    const SyncWs w = sync_ws(const_cast<void *>(workspace), s->info.n_subseq);
    return hipMemcpyAsync(gap_out, w.gap_s, s->info.n_subseq, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(hip_stream)) == hipSuccess
               ? HD_OK
               : HD_ERR_DEVICE;
}

namespace {

// Workspace layout of a batch: the status header, then the stream
// descriptors.  Both travel in one upload, so the status word starts zeroed
// (word 1, the slot count, is 0: the batch kernel ORs into word 0).
struct BatchLayout {
    size_t desc, total;
};

hd_status batch_layout(uint32_t n, BatchLayout *L)
{
    L->desc = kWsHeader;
    L->total = kWsHeader + align_up(sizeof(BatchStreamDev) * size_t(n), 256);
    return HD_OK;
}

// Pinned host staging for per-call descriptors.  A buffer is reused only
// after the event recorded behind its last upload has completed, so uploads
// never wait for the host and never race with earlier calls.
struct StagingBuf {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
};

std::mutex g_stage_mu;
std::vector<StagingBuf *> g_stage;

StagingBuf *staging_acquire(size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (StagingBuf *b : g_stage) {
        if (b->busy && hipEventQuery(b->done) == hipSuccess)
            b->busy = false;
        if (!b->busy && b->cap >= bytes) {
            b->busy = true;
            return b;
        }
    }
    StagingBuf *b = new StagingBuf();
    if (hipHostMalloc(&b->host, bytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return nullptr;
    }
    b->cap = bytes;
    b->busy = true;
    g_stage.push_back(b);
    return b;
}

// The batch kernel for a set of table formats; `small`: every subsequence
// of the batch has at most 32 * kSmallUnits bits (smaller tile-input
// registers, and the entry-log replay for pair-format streams).
template <uint32_t MAXU>
const void *batch_kernel_of(int formats)
{
    switch (formats) {
    case kBatchPairOnly: return reinterpret_cast<const void *>(&k_decode_batch<kBatchPairOnly, MAXU>);
    case kBatchWideOnly: return reinterpret_cast<const void *>(&k_decode_batch<kBatchWideOnly, MAXU>);
    default: return reinterpret_cast<const void *>(&k_decode_batch<kBatchMixed, MAXU>);
    }
}

const void *batch_kernel(int formats, bool small)
{
    return small ? batch_kernel_of<kSmallUnits>(formats) : batch_kernel_of<kMaxUnitsPerLane>(formats);
}

template <int FORMATS, uint32_t MAXU>
hd_status launch_batch_as(const BatchArgs &a, uint32_t wpg, uint32_t lds, uint32_t grid, hipStream_t stream)
{
    if (!allow_full_lds(reinterpret_cast<const void *>(&k_decode_batch<FORMATS, MAXU>)))
        return HD_ERR_DEVICE;
    hipLaunchKernelGGL((k_decode_batch<FORMATS, MAXU>), dim3(grid), dim3(wpg * 64), lds, stream, a);
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}

template <uint32_t MAXU>
hd_status launch_batch_of(const BatchArgs &a, int formats, uint32_t wpg, uint32_t lds, uint32_t grid,
                          hipStream_t stream)
{
    switch (formats) {
    case kBatchPairOnly: return launch_batch_as<kBatchPairOnly, MAXU>(a, wpg, lds, grid, stream);
    case kBatchWideOnly: return launch_batch_as<kBatchWideOnly, MAXU>(a, wpg, lds, grid, stream);
    default: return launch_batch_as<kBatchMixed, MAXU>(a, wpg, lds, grid, stream);
    }
}

hd_status launch_batch(const BatchArgs &a, int formats, bool small, uint32_t wpg, uint32_t lds, uint32_t grid,
                       hipStream_t stream)
{
    return small ? launch_batch_of<kSmallUnits>(a, formats, wpg, lds, grid, stream)
                 : launch_batch_of<kMaxUnitsPerLane>(a, formats, wpg, lds, grid, stream);
}


}  // namespace

extern "C" hd_status hd_decode_batch_workspace_size(const hd_dstream *streams, uint32_t n_streams,
                                                    hd_mode m, size_t *bytes)
{
    if (!bytes || (n_streams && !streams))
        return HD_ERR_ARG;
    if (m != HD_MODE_GAP)
        return HD_ERR_UNSUPPORTED;
    for (uint32_t i = 0; i < n_streams; ++i) {
        hd_status st = check_stream(&streams[i], m);
        if (st == HD_OK && sym_bytes(streams[i].info) != 2)
            st = HD_ERR_UNSUPPORTED;
        if (st != HD_OK)
            return st;
    }
    BatchLayout L;
    hd_status st = batch_layout(n_streams, &L);
    if (st != HD_OK)
        return st;
    *bytes = L.total;
    return HD_OK;
}

namespace {

// Batched decode: streams of at least this many symbols get their own decode
// launch (a persistent grid of the single-stream kernel is then mostly full).
constexpr uint64_t kBatchSoloSymbols = uint64_t(1) << 23;

hd_status decode_batch_impl(const hd_dstream *streams, uint32_t n_streams, uint16_t *const *outs, hd_mode m,
                            const hd_tune *per_stream, void *workspace, size_t ws_bytes, void *hip_stream,
                            uint32_t *direct)
{
    if (n_streams == 0)
        return HD_OK;
    if (!streams || !outs || !workspace || reinterpret_cast<uintptr_t>(workspace) % 256)
        return HD_ERR_ARG;
    size_t need = 0;
    hd_status st = hd_decode_batch_workspace_size(streams, n_streams, m, &need);
    if (st != HD_OK)
        return st;
    if (ws_bytes < need)
        return HD_ERR_ARG;
    const DeviceInfo *dev = device_info();
    if (!dev)
        return HD_ERR_DEVICE;
    BatchLayout L;
    st = batch_layout(n_streams, &L);
    if (st != HD_OK)
        return st;
    char *ws = static_cast<char *>(workspace);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);

    // Streams of at least kBatchSoloSymbols fill the device on their own:
    // each gets the single-stream decode launch with its own plan (table
    // format, registers, staging and occupancy of that stream), enqueued
    // first.  The rest share one persistent launch, whose LDS layout reserves
    // the largest table, subsequence and staging among them; its waves per
    // workgroup and workgroups per CU come from per_stream[0] (zero: the most
    // resident wavefronts that layout allows).
    uint32_t S_alloc = 32, stage_alloc = 256, k1_alloc = 1, n_pair = 0, auto_max = 0;
    std::vector<uint32_t> stage(n_streams);
    std::vector<bool> given(n_streams);
    std::vector<uint32_t> shared, solo;
    for (uint32_t i = 0; i < n_streams; ++i) {
        const hd_stream_info &si = streams[i].info;
        const hd_tune *tu = per_stream ? &per_stream[i] : nullptr;
        given[i] = tu && tu->stage_symbols;
        stage[i] = given[i] ? tu->stage_symbols : auto_stage_for(si);
        if (stage[i] < 256 || stage[i] > 16384 || stage[i] % 64)
            return HD_ERR_ARG;
        if ((si.n_symbols && !outs[i]) || reinterpret_cast<uintptr_t>(outs[i]) % 16 ||
            reinterpret_cast<uintptr_t>(streams[i].words) % 16)
            return HD_ERR_ARG;
        if (64 % si.chunk_subseqs)
            return HD_ERR_UNSUPPORTED;
        if (si.n_symbols >= kBatchSoloSymbols) {
            solo.push_back(i);
            continue;
        }
        shared.push_back(i);
        if (!given[i])
            auto_max = std::max(auto_max, stage[i]);
        S_alloc = std::max(S_alloc, si.subseq_bits);
        if (given[i])
            stage_alloc = std::max(stage_alloc, stage[i]);
        k1_alloc = std::max(k1_alloc, streams[i].table->k1);
        n_pair += streams[i].table->pair ? 1u : 0u;
    }
    if (auto_max) {
        // default staging: the largest need of the batch, capped where it
        // would cost occupancy for everyone -- at the larger of the size that
        // keeps 16 wavefronts resident per CU and the symbol-weighted median
        // need (streams above the cap decode their larger tiles in passes)
        std::vector<std::pair<uint32_t, uint64_t>> need;
        uint64_t total = 0;
        for (uint32_t i : shared)
            if (!given[i]) {
                need.emplace_back(stage[i], streams[i].info.n_symbols);
                total += streams[i].info.n_symbols;
            }
        std::sort(need.begin(), need.end());
        uint32_t median = need.back().first;
        uint64_t acc = 0;
        for (const auto &nd : need)
            if ((acc += nd.second) * 2 >= total) {
                median = nd.first;
                break;
            }
        const uint32_t cap = std::max(median, stage_for_waves(table_lds_bytes(k1_alloc), S_alloc, 16, dev));
        const uint32_t use = std::min(auto_max, cap);
        for (uint32_t i : shared)
            if (!given[i])
                stage[i] = std::min(stage[i], use);
        stage_alloc = std::max(stage_alloc, use);
    }
    const uint32_t n_shared = static_cast<uint32_t>(shared.size());
    const uint32_t table = table_lds_bytes(k1_alloc), area = wave_area_bytes(S_alloc, stage_alloc);
    const hd_tune *t0 = per_stream ? &per_stream[0] : nullptr;
    const int formats = n_pair == n_shared ? kBatchPairOnly : n_pair == 0 ? kBatchWideOnly : kBatchMixed;
    const bool small = S_alloc <= 32 * kSmallUnits;
    const void *func = batch_kernel(formats, small);
    const uint32_t reg_cap = reg_waves_per_cu(func);
    const uint32_t wpg = t0 && t0->waves_per_group ? t0->waves_per_group
                                                   : occupancy_wpg(table, area, dev, nullptr, reg_cap, func);
    if (wpg == 0)
        return HD_ERR_UNSUPPORTED;
    if (wpg > kMaxWavesPerGroup)
        return HD_ERR_ARG;
    const uint32_t lds = table + wpg * area;
    if (lds > dev->lds_per_block)
        return HD_ERR_UNSUPPORTED;
    uint32_t fit = std::max<uint32_t>(1, std::min<uint32_t>(static_cast<uint32_t>(lds_cu_usable(dev) / lds),
                                                            std::min<uint32_t>(reg_cap, 4 * kSimdWaveCap) / wpg));
    const int nb = resident_groups(func, wpg * 64, lds);
    if (nb > 0)
        fit = std::min<uint32_t>(fit, static_cast<uint32_t>(nb));
    if (t0 && t0->groups_per_cu)
        fit = std::min(fit, t0->groups_per_cu);

    std::vector<BatchStreamDev> d(n_shared);
    uint64_t items = 0;
    for (uint32_t q = 0; q < n_shared; ++q) {
        const uint32_t i = shared[q];
        const hd_dstream &s = streams[i];
        const hd_stream_info &si = s.info;
        BatchStreamDev &b = d[q];
        b.sd.words = s.words;
        b.sd.gap = s.gap;
        b.sd.chunk_off = s.chunk_offsets;
        b.sd.out = outs[i];
        b.sd.n = si.n_symbols;
        b.sd.B = si.n_bits;
        b.sd.K = si.n_subseq;
        b.sd.M = si.n_chunks;
        b.sd.n_words = si.n_words;
        b.sd.S = si.subseq_bits;
        b.sd.last_bits = si.n_subseq ? static_cast<uint32_t>(si.n_bits - (si.n_subseq - 1) * si.subseq_bits) : 0u;
        b.sd.Cl = chunk_log2(si.chunk_subseqs);
        b.sd.stage = stage[i];
        b.tab = view_of(s.table);
        b.pair = s.table->pair ? 1 : 0;
        b.pad = 0;
        b.ntiles = ceil_div(si.n_subseq, 64);
        b.item0 = items;
        items += ceil_div(b.ntiles, wpg);
    }

    // upload the zeroed status header and the descriptors through pinned
    // staging, in one copy
    const size_t up = L.total;
    StagingBuf *sb = staging_acquire(up);
    if (!sb)
        return HD_ERR_NOMEM;
    char *h = static_cast<char *>(sb->host);
    std::memset(h, 0, up);
    std::memcpy(h + L.desc, d.data(), sizeof(BatchStreamDev) * n_shared);
    if (hipMemcpyAsync(ws, h, up, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipEventRecord(sb->done, stream) != hipSuccess) {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        sb->busy = false;
        return HD_ERR_DEVICE;
    }
    uint32_t *status = reinterpret_cast<uint32_t *>(ws);
    // the large streams, after the upload that zeroes the status word: each
    // wavefront that met an error ORs its bits into that word (or, for the
    // server, stores them into its pinned word)
    for (uint32_t i : solo) {
        hd_tune tu{};
        if (given[i])
            tu.stage_symbols = stage[i];
        st = run_decode_kernel(&streams[i], outs[i], HD_MODE_GAP, given[i] ? &tu : nullptr, nullptr,
                               direct ? direct : status, stream, direct == nullptr);
        if (st != HD_OK)
            return st;
    }
    if (items == 0)
        return HD_OK;
    BatchArgs a;
    a.streams = reinterpret_cast<const BatchStreamDev *>(ws + L.desc);
    a.n_streams = n_shared;
    a.n_items = items;
    a.status = direct ? direct : status;
    a.direct = direct ? 1u : 0u;
    a.S_alloc = S_alloc;
    a.stage_alloc = stage_alloc;
    a.k1_alloc = k1_alloc;
    const uint32_t grid = static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(items, uint64_t(dev->cus) * fit)));
    return launch_batch(a, formats, small, wpg, lds, grid, stream);
}

}  // namespace

extern "C" hd_status hd_decode_batch(const hd_dstream *streams, uint32_t n_streams,
                                     uint16_t *const *outs, hd_mode m, const hd_tune *per_stream,
                                     void *workspace, size_t ws_bytes, void *hip_stream)
{
    return decode_batch_impl(streams, n_streams, outs, m, per_stream, workspace, ws_bytes, hip_stream, nullptr);
}

hd_status hd::decode_batch_direct(const hd_dstream *streams, uint32_t n_streams, uint16_t *const *outs,
                                  uint32_t *status_word, void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!status_word)
        return HD_ERR_ARG;
    return decode_batch_impl(streams, n_streams, outs, HD_MODE_GAP, nullptr, workspace, ws_bytes, hip_stream,
                             status_word);
}

extern "C" hd_status hd_autotune(const hd_dstream *sample, hd_mode m, void *out, void *workspace,
                                 size_t ws_bytes, void *hip_stream, hd_tune *best, float *best_ms)
{
    if (!best)
        return HD_ERR_ARG;
    hd_status st = check_call(sample, m, nullptr, workspace, ws_bytes);
    if (st != HD_OK)
        return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const uint32_t base = auto_stage_for(sample->info);
    const double mult[] = {0.5, 0.75, 1.0, 1.5, 2.0};
    const uint32_t wpgs[] = {0, 4, 8, 16};     // 0: the occupancy choice for each staging size
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return HD_ERR_DEVICE;
    float best_t = 0.f;
    bool have = false;
    // the output-index phase does not depend on the tune: run it once
    st = hd_decode_prepare(sample, m, nullptr, workspace, ws_bytes, hip_stream);
    for (uint32_t w : wpgs) {
        for (double f : mult) {
            if (st != HD_OK)
                break;
            uint32_t stage = static_cast<uint32_t>(base * f);
            stage = std::min<uint32_t>(16384, std::max<uint32_t>(256, (stage + 63) / 64 * 64));
            hd_tune t{w, stage, 0, 0};
            Plan p;
            if (make_plan(sample, &t, &p) != HD_OK)
                continue;                               // LDS request too large
            if (w == 0 && (p.wpg == 4 || p.wpg == 8 || p.wpg == 16))
                continue;                               // timed with the fixed sizes
            t.waves_per_group = p.wpg;
            float times[3];
            hd_status rs = hd_decode_run(sample, out, m, &t, workspace, ws_bytes, hip_stream);   // warm-up
            for (int r = 0; r < 3 && rs == HD_OK; ++r) {
                if (hipEventRecord(e0, stream) != hipSuccess) {
                    rs = HD_ERR_DEVICE;
                    break;
                }
                rs = hd_decode_run(sample, out, m, &t, workspace, ws_bytes, hip_stream);
                if (rs == HD_OK && hipEventRecord(e1, stream) != hipSuccess)
                    rs = HD_ERR_DEVICE;
                if (rs != HD_OK)
                    break;
                if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&times[r], e0, e1) != hipSuccess)
                    rs = HD_ERR_DEVICE;
            }
            if (rs != HD_OK) {
                st = rs;
                break;
            }
            std::sort(times, times + 3);
            if (!have || times[1] < best_t) {
                best_t = times[1];
                *best = t;
                have = true;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HD_OK)
        return st;
    if (!have)
        return HD_ERR_UNSUPPORTED;
    if (best_ms)
        *best_ms = best_t;
    return HD_OK;
}

extern "C" uint32_t hd_decode_status_bits(const void *workspace, void *hip_stream)
{
    if (!workspace)
        return 0xffffffffu;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (hipStreamSynchronize(stream) != hipSuccess)
        return 0xffffffffu;
    // header word 0, OR-ed with the per-wavefront slots the last decode
    // kernel wrote (word 1 counts them; 0 for batches, reconstruction and
    // encoding, which report in word 0 alone)
    uint32_t head[2] = {0, 0};
    if (hipMemcpy(head, workspace, sizeof(head), hipMemcpyDeviceToHost) != hipSuccess)
        return 0xffffffffu;
    if (head[1] > kMaxSlots)
        return 0xffffffffu;
    uint32_t v = head[0];
    if (head[1]) {
        std::vector<uint32_t> slots(head[1]);
        if (hipMemcpy(slots.data(), static_cast<const char *>(workspace) + kWsHeader, 4 * size_t(head[1]),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return 0xffffffffu;
        for (uint32_t e : slots)
            v |= e;
    }
    return v == 0xffffffffu ? v & ~0x80000000u : v;
}

extern "C" hd_status hd_decode_status(const void *workspace, void *hip_stream)
{
    if (!workspace)
        return HD_ERR_ARG;
    const uint32_t v = hd_decode_status_bits(workspace, hip_stream);
    if (v == 0xffffffffu)
        return HD_ERR_DEVICE;
    return v ? HD_ERR_CORRUPT : HD_OK;
}

// ------------------------------------------------------------------------
// Allocation-free decode
// ------------------------------------------------------------------------
//
// hd_decode with its workspace in a fixed device array.  Host code never
// passes the array's name to a kernel: in host code the name is only a
// stand-in for the symbol, so the device address of each GPU's copy is looked
// up once (hipGetSymbolAddress, with that device current) and kept per device.

namespace {

constexpr size_t kScratchBytes = HD_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[64];

// The current device's copy of the array (nullptr when the lookup fails).
void *scratch_of_current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

// One workgroup: the status word of a decode workspace, header word 0 OR the
// slots the last decode kernel wrote (word 1 counts them), stored to *out.
__global__ __launch_bounds__(256) void k_fold_status(const uint32_t *ws, uint32_t *out)
{
    __shared__ uint32_t acc[4];
    const uint32_t ns = ws[1];
    uint32_t v = 0;
    if (ns > kMaxSlots) {
        v = 0xffffffffu;                              // an unreadable status
    } else {
        const uint32_t *slots = ws + kWsHeader / 4;
        for (uint32_t i = threadIdx.x; i < ns; i += blockDim.x)
            v |= slots[i];
        if (threadIdx.x == 0)
            v |= ws[0];
    }
    v = wave_or(v);
    if ((threadIdx.x & 63) == 0)
        acc[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t r = acc[0] | acc[1] | acc[2] | acc[3];
        // all ones means "unreadable"; status bits alone never reach bit 31
        *out = ns > kMaxSlots ? r : (r & 0x7fffffffu);
    }
}

}  // namespace

extern "C" hd_status hd_decode_noalloc(const hd_dstream *s, void *out, hd_mode m, const hd_tune *tune,
                                       uint32_t *status, void *hip_stream)
{
    hd_status st = check_stream(s, m);
    if (st != HD_OK)
        return st;
    if (!status || reinterpret_cast<uintptr_t>(status) % 4 != 0)
        return HD_ERR_ARG;
    size_t need = 0;
    st = hd_decode_workspace_size(s, m, tune, &need);
    if (st != HD_OK)
        return st;
    if (need > kScratchBytes)
        return HD_ERR_UNSUPPORTED;
    void *ws = scratch_of_current_device();
    if (!ws)
        return HD_ERR_DEVICE;
    st = hd_decode(s, out, m, tune, ws, kScratchBytes, hip_stream);
    if (st != HD_OK)
        return st;
    hipLaunchKernelGGL(k_fold_status, dim3(1), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<const uint32_t *>(ws), status);
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}
