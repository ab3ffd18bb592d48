// Host half of the library: codebook construction and the reference encoder.
//
// Huffman codes give frequent fixed-length input symbols short prefix-free
// codewords (Sec. II-B).  The paper leaves codebook construction to its
// encoder; this library builds an optimal code under a length limit L with a
// counting form of package-merge, and assigns canonical codes so the decoder
// can use a compact lookup table (first level + per-length limits).
//
// The encoder writes the stream format described in include/hd.h: 32-bit
// units (Sec. III-B), one gap byte per subsequence (Sec. III-C) and the output
// index of every chunk's first codeword (Sec. III-B, step 3, stored).
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "hd.h"

namespace {

struct Leaf {
    uint64_t w;
    uint32_t sym;
};

// Package-merge, counting form.  Level L holds the symbols ranked by
// (count, symbol).  Level d < L holds the same symbols merged with the pairs
// of level d+1 (a symbol ahead of a pair of equal weight).  Taking the first
// 2m-2 items of level 1 and, recursively, the first 2p items of level d+1 for
// the p pairs taken at level d, the symbols taken at every level are a prefix
// of the ranking; a symbol's length is the number of levels whose prefix
// covers it.
hd_status lengths_package_merge(const uint64_t *hist, uint32_t A, uint32_t L, uint8_t *len)
{
    std::vector<Leaf> leaves;
    leaves.reserve(A);
    for (uint32_t s = 0; s < A; ++s) {
        len[s] = 0;
        if (hist[s])
            leaves.push_back({hist[s], s});
    }
    const uint32_t m = static_cast<uint32_t>(leaves.size());
    if (m == 0)
        return HD_OK;
    if (m == 1) {
        len[leaves[0].sym] = 1;
        return HD_OK;
    }
    if (L < 32 && m > (1u << L))
        return HD_ERR_INFEASIBLE;
    std::sort(leaves.begin(), leaves.end(), [](const Leaf &a, const Leaf &b) {
        return a.w != b.w ? a.w < b.w : a.sym < b.sym;
    });

    // is_pair[d][i]: item i of level d (d = 1..L) is a pair.  Level weights
    // are only needed for the level being built.
    std::vector<std::vector<uint8_t>> is_pair(L + 1);
    std::vector<uint64_t> cur(m), nxt;
    for (uint32_t i = 0; i < m; ++i)
        cur[i] = leaves[i].w;
    is_pair[L].assign(m, 0);
    for (uint32_t d = L - 1; d >= 1; --d) {
        const size_t npairs = cur.size() / 2;
        nxt.clear();
        nxt.reserve(m + npairs);
        is_pair[d].clear();
        is_pair[d].reserve(m + npairs);
        size_t li = 0, pi = 0;
        while (li < m || pi < npairs) {
            const uint64_t pw = pi < npairs ? cur[2 * pi] + cur[2 * pi + 1] : 0;
            if (pi >= npairs || (li < m && leaves[li].w <= pw)) {
                nxt.push_back(leaves[li++].w);
                is_pair[d].push_back(0);
            } else {
                nxt.push_back(pw);
                is_pair[d].push_back(1);
                ++pi;
            }
        }
        cur.swap(nxt);
        if (d == 1)
            break;
    }
    // Walk the selection down the levels.
    std::vector<uint32_t> depth(m, 0);
    uint64_t take = 2ull * m - 2;
    for (uint32_t d = 1; d <= L && take > 0; ++d) {
        const std::vector<uint8_t> &ip = is_pair[d];
        if (take > ip.size())
            return HD_ERR_INFEASIBLE;
        uint64_t pairs = 0, singles = 0;
        for (uint64_t i = 0; i < take; ++i) {
            if (ip[i])
                ++pairs;
            else
                ++singles;
        }
        for (uint64_t i = 0; i < singles; ++i)
            ++depth[i];
        take = 2 * pairs;
    }
    for (uint32_t i = 0; i < m; ++i)
        len[leaves[i].sym] = static_cast<uint8_t>(depth[i]);
    return HD_OK;
}

// Canonical assignment by per-length counts: the first code of length l is
// (first code of length l-1 + number of codes of length l-1) << 1, and codes
// of one length are handed out in increasing symbol order.
hd_status canonical_from_lengths(const uint8_t *len, uint32_t A, uint32_t L, uint32_t *codes)
{
    uint64_t bl[34] = {0};
    for (uint32_t s = 0; s < A; ++s) {
        if (len[s] > L)
            return HD_ERR_ARG;
        bl[len[s]]++;
    }
    bl[0] = 0;
    uint64_t next[34] = {0};
    uint64_t c = 0;
    for (uint32_t l = 1; l <= 32; ++l) {
        c = (c + bl[l - 1]) << 1;
        next[l] = c;
    }
    for (uint32_t s = 0; s < A; ++s) {
        const uint32_t l = len[s];
        if (l == 0) {
            codes[s] = 0;
            continue;
        }
        const uint64_t v = next[l]++;
        if (v >> l)
            return HD_ERR_ARG;                  // lengths oversubscribe the code space
        codes[s] = static_cast<uint32_t>(v);
    }
    return HD_OK;
}

// Symbol width of a layout (0 reads as 2) and whether alphabet A fits it.
uint32_t layout_width(const hd_layout *lay) { return lay->symbol_bytes ? lay->symbol_bytes : 2u; }

bool width_fits(uint32_t w, uint32_t A)
{
    return A != 0 && ((w == 1 && A <= 256u) || (w == 2 && A <= 65536u) || (w == 4 && A <= HD_MAX_ALPHABET));
}

template <typename T>
hd_status encode_as(const T *syms, uint64_t n, const uint8_t *lengths, const uint32_t *codes, uint32_t A,
                    uint32_t L, const hd_layout *lay, uint32_t *words, uint64_t words_cap, uint8_t *gap,
                    uint64_t gap_cap, uint64_t *chunk_offsets, uint64_t chunk_cap, hd_stream_info *info);

}  // namespace

extern "C" hd_status hd_canonical_codes_internal(const uint8_t *len, uint32_t A, uint32_t L,
                                                 uint32_t *codes)
{
    return canonical_from_lengths(len, A, L, codes);
}

extern "C" hd_status hd_build_codebook(const uint64_t *hist, uint32_t A, uint32_t L,
                                       uint8_t *lengths, uint32_t *codes)
{
    if (!hist || !lengths || !codes || A == 0 || A > HD_MAX_ALPHABET || L == 0 || L > 32)
        return HD_ERR_ARG;
    try {
        hd_status st = lengths_package_merge(hist, A, L, lengths);
        if (st != HD_OK)
            return st;
        return canonical_from_lengths(lengths, A, L, codes);
    } catch (const std::bad_alloc &) {
        return HD_ERR_NOMEM;
    } catch (...) {
        return HD_ERR_ARG;
    }
}

extern "C" hd_status hd_encode_ref(const void *syms, uint64_t n, const uint8_t *lengths,
                                   const uint32_t *codes, uint32_t A, uint32_t L,
                                   const hd_layout *lay, uint32_t *words, uint64_t words_cap,
                                   uint8_t *gap, uint64_t gap_cap, uint64_t *chunk_offsets,
                                   uint64_t chunk_cap, hd_stream_info *info)
{
    if (!lengths || !codes || !lay || !info || (n && !syms))
        return HD_ERR_ARG;
    const uint32_t w = layout_width(lay);
    if (!width_fits(w, A) || L == 0 || L > 32)
        return HD_ERR_ARG;
    if (w == 1)
        return encode_as(static_cast<const uint8_t *>(syms), n, lengths, codes, A, L, lay, words, words_cap, gap,
                         gap_cap, chunk_offsets, chunk_cap, info);
    if (w == 2)
        return encode_as(static_cast<const uint16_t *>(syms), n, lengths, codes, A, L, lay, words, words_cap, gap,
                         gap_cap, chunk_offsets, chunk_cap, info);
    return encode_as(static_cast<const uint32_t *>(syms), n, lengths, codes, A, L, lay, words, words_cap, gap,
                     gap_cap, chunk_offsets, chunk_cap, info);
}

namespace {

template <typename T>
hd_status encode_as(const T *syms, uint64_t n, const uint8_t *lengths, const uint32_t *codes, uint32_t A,
                    uint32_t L, const hd_layout *lay, uint32_t *words, uint64_t words_cap, uint8_t *gap,
                    uint64_t gap_cap, uint64_t *chunk_offsets, uint64_t chunk_cap, hd_stream_info *info)
{
    const uint32_t S = lay->subseq_bits, C = lay->chunk_subseqs;
    if (S < 32 || S % 32 != 0 || C == 0)
        return HD_ERR_ARG;
    for (uint32_t s = 0; s < A; ++s)
        if (lengths[s] > L)
            return HD_ERR_ARG;

    uint64_t B = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t s = syms[i];
        if (s >= A || lengths[s] == 0)
            return HD_ERR_SYMBOL;
        B += lengths[s];
    }
    const uint64_t K = (B + S - 1) / S;
    const uint64_t M = (K + C - 1) / C;
    const uint64_t NW = K * (S / 32) + 2;
    info->n_symbols = n;
    info->n_bits = B;
    info->n_words = NW;
    info->n_subseq = K;
    info->n_chunks = M;
    info->subseq_bits = S;
    info->chunk_subseqs = C;
    info->alphabet_size = A;
    info->max_len = L;
    info->symbol_bytes = layout_width(lay);
    info->reserved = 0;
    if (!words)
        return HD_OK;
    if (words_cap < NW || gap_cap < K || chunk_cap < M + 1 || !chunk_offsets || (K && !gap))
        return HD_ERR_ARG;

    // chunk_offsets[c]: codewords that start before chunk c (filled as each
    // chunk's first codeword goes by; chunks without one take the next)
    const uint64_t chunk_bits = static_cast<uint64_t>(S) * C;
    uint64_t next_chunk = 0;
    uint64_t acc = 0;       // pending bits, right-aligned
    uint32_t nacc = 0;      // number of pending bits (< 32 between symbols)
    uint64_t wi = 0;        // next unit to write
    uint64_t pos = 0;       // bit position of the current codeword
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t s = syms[i];
        const uint32_t l = lengths[s];
        // Subsequence boundaries this codeword starts on or straddles: the
        // first codeword start at or after each is pos (on) or pos+l (inside).
        const uint64_t end = pos + l;
        uint64_t b = (pos + S - 1) / S * S;
        if (b == pos) {
            gap[b / S] = 0;
            b += S;
        }
        for (; b < end; b += S)
            gap[b / S] = static_cast<uint8_t>(end - b);
        for (; next_chunk <= pos / chunk_bits; ++next_chunk)
            chunk_offsets[next_chunk] = i;

        acc = (acc << l) | codes[s];
        nacc += l;
        while (nacc >= 32) {
            nacc -= 32;
            words[wi++] = static_cast<uint32_t>(acc >> nacc);
        }
        acc &= (nacc ? ((uint64_t(1) << nacc) - 1) : 0);
        pos = end;
    }
    for (; next_chunk <= M; ++next_chunk)
        chunk_offsets[next_chunk] = n;
    if (nacc)
        words[wi++] = static_cast<uint32_t>(acc << (32 - nacc));
    for (; wi < NW; ++wi)
        words[wi] = 0;
    return HD_OK;
}

}  // namespace

extern "C" hd_status hd_stream_layout(uint64_t n_symbols, uint64_t n_bits, uint32_t A, uint32_t L,
                                      const hd_layout *lay, hd_stream_info *info)
{
    if (!lay || !info || !width_fits(layout_width(lay), A) || L == 0 || L > 32)
        return HD_ERR_ARG;
    const uint32_t S = lay->subseq_bits, C = lay->chunk_subseqs;
    if (S < 32 || S % 32 != 0 || C == 0)
        return HD_ERR_ARG;
    if (n_bits < n_symbols || static_cast<unsigned __int128>(n_bits) > static_cast<unsigned __int128>(L) * n_symbols)
        return HD_ERR_CORRUPT;
    const uint64_t K = (n_bits + S - 1) / S;
    info->n_symbols = n_symbols;
    info->n_bits = n_bits;
    info->n_subseq = K;
    info->n_chunks = (K + C - 1) / C;
    info->n_words = K * (S / 32) + 2;
    info->subseq_bits = S;
    info->chunk_subseqs = C;
    info->alphabet_size = A;
    info->max_len = L;
    info->symbol_bytes = layout_width(lay);
    info->reserved = 0;
    return HD_OK;
}

extern "C" const char *hd_status_str(hd_status s)
{
    switch (s) {
    case HD_OK: return "ok";
    case HD_ERR_ARG: return "invalid argument";
    case HD_ERR_INFEASIBLE: return "more used symbols than the length limit allows";
    case HD_ERR_SYMBOL: return "symbol out of range or without a codeword";
    case HD_ERR_CORRUPT: return "stream inconsistent with its codebook or metadata";
    case HD_ERR_NOMEM: return "out of memory";
    case HD_ERR_DEVICE: return "HIP runtime error";
    case HD_ERR_UNSUPPORTED: return "unsupported input";
    }
    return "unknown status";
}
