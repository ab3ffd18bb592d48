// Host-code check under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Built by tests/test_sanitize_cpu.py with g++ from the library's host-only
// source (codebook construction, reference encoder, stream layout) and the
// C oracle, then run: every call below must stay in bounds and free of
// undefined behaviour, and the two sides must agree (codebook lengths and
// codes, encoded words, gap array, chunk offsets) on random inputs and on
// the edge cases (one used symbol, empty input, the length limit binding,
// infeasible limits, counts near 2^40, bad arguments).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "hd.h"

extern "C" {
int hdref_histogram(const uint16_t *x, uint64_t n, uint32_t A, uint64_t *cnt);
int hdref_code_lengths(const uint64_t *cnt, uint32_t A, uint32_t L, uint8_t *len);
int hdref_canonical_codes(const uint8_t *len, uint32_t A, uint32_t *code);
int hdref_encode(const uint16_t *x, uint64_t n, const uint8_t *len, const uint32_t *code, uint32_t A, uint32_t S,
                 uint32_t C, uint32_t *words, uint64_t words_cap, uint8_t *gap, uint64_t gap_cap,
                 uint32_t *chunk_counts, uint64_t chunk_cap, uint64_t *info);
int hdref_decode(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n, const uint8_t *len,
                 const uint32_t *code, uint32_t A, uint16_t *out);
int hdref_selfsync(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n, const uint8_t *len,
                   const uint32_t *code, uint32_t A, uint32_t S, uint8_t *sync_gap, uint32_t *counts,
                   uint32_t *sync_bits);
int hdref_gap_backward(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n, const uint8_t *len,
                       const uint32_t *code, uint32_t A, uint32_t S, int32_t *gapb, uint32_t *counts_b);
}

static int g_fail = 0;
#define CHECK(c)                                                                                        \
    do {                                                                                                \
        if (!(c)) {                                                                                     \
            std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c);                           \
            ++g_fail;                                                                                   \
        }                                                                                               \
    } while (0)

static std::vector<uint16_t> geometric_symbols(std::mt19937_64 &rng, uint64_t n, uint32_t A, double r)
{
    std::geometric_distribution<int64_t> g(1.0 - r);
    std::vector<uint16_t> x(n);
    for (auto &v : x) {
        int64_t d = int64_t(A / 2) + g(rng) - g(rng);
        v = (d < 0 || d >= int64_t(A)) ? 0 : uint16_t(d);
    }
    return x;
}

// One stream through both encoders and the oracle's decoders.
static void round_trip(const std::vector<uint16_t> &x, uint32_t A, uint32_t L, uint32_t S, uint32_t C)
{
    std::vector<uint64_t> h1(A), h2(A, 0);
    CHECK(hdref_histogram(x.data(), x.size(), A, h1.data()) == 0);
    for (uint16_t v : x)
        h2[v]++;
    CHECK(h1 == h2);
    std::vector<uint8_t> len(A), len2(A);
    std::vector<uint32_t> code(A), code2(A);
    const int rc = hdref_code_lengths(h1.data(), A, L, len.data());
    const hd_status st = hd_build_codebook(h1.data(), A, L, len2.data(), code2.data());
    if (rc != 0) {
        CHECK(rc == -2 && st == HD_ERR_INFEASIBLE);
        return;
    }
    CHECK(st == HD_OK);
    CHECK(hdref_canonical_codes(len.data(), A, code.data()) == 0);
    CHECK(len == len2);
    CHECK(code == code2);

    uint64_t info[4];
    CHECK(hdref_encode(x.data(), x.size(), len.data(), code.data(), A, S, C, nullptr, 0, nullptr, 0, nullptr, 0,
                       info) == 0);
    const uint64_t B = info[0], NW = info[1], K = info[2], M = info[3];
    std::vector<uint32_t> w1(NW), cc(M + 1);
    std::vector<uint8_t> g1(K + 1);
    CHECK(hdref_encode(x.data(), x.size(), len.data(), code.data(), A, S, C, w1.data(), NW, g1.data(), K, cc.data(),
                       M, info) == 0);

    hd_layout lay{S, C};
    hd_stream_info si;
    CHECK(hd_encode_ref(x.data(), x.size(), len.data(), code.data(), A, L, &lay, nullptr, 0, nullptr, 0, nullptr, 0,
                        &si) == HD_OK);
    CHECK(si.n_bits == B && si.n_words == NW && si.n_subseq == K && si.n_chunks == M);
    hd_stream_info si2;
    CHECK(hd_stream_layout(x.size(), B, A, L, &lay, &si2) == HD_OK || x.empty());
    std::vector<uint32_t> w2(NW);
    std::vector<uint8_t> g2(K + 1);
    std::vector<uint64_t> off(M + 1);
    CHECK(hd_encode_ref(x.data(), x.size(), len.data(), code.data(), A, L, &lay, w2.data(), NW, g2.data(), K,
                        off.data(), M + 1, &si) == HD_OK);
    CHECK(w1 == w2);
    CHECK(K == 0 || std::memcmp(g1.data(), g2.data(), K) == 0);
    uint64_t acc = 0;
    for (uint64_t c = 0; c < M; ++c) {
        CHECK(off[c] == acc);
        acc += cc[c];
    }
    CHECK(off[M] == x.size());
    // a short buffer is refused
    if (NW > 1)
        CHECK(hd_encode_ref(x.data(), x.size(), len.data(), code.data(), A, L, &lay, w2.data(), NW - 1, g2.data(),
                            K, off.data(), M + 1, &si) == HD_ERR_ARG);

    std::vector<uint16_t> y(x.size() + 1);
    CHECK(hdref_decode(w1.data(), NW, B, x.size(), len.data(), code.data(), A, y.data()) == 0);
    CHECK(x.empty() || std::memcmp(x.data(), y.data(), 2 * x.size()) == 0);
    std::vector<uint8_t> sg(K + 1);
    std::vector<uint32_t> cnt(K + 1), sb(K + 1);
    CHECK(hdref_selfsync(w1.data(), NW, B, x.size(), len.data(), code.data(), A, S, sg.data(), cnt.data(),
                         sb.data()) == 0);
    CHECK(K == 0 || std::memcmp(sg.data(), g1.data(), K) == 0);
    std::vector<int32_t> gb(K + 1);
    CHECK(hdref_gap_backward(w1.data(), NW, B, x.size(), len.data(), code.data(), A, S, gb.data(), cnt.data()) ==
          0);
}

int main()
{
    std::mt19937_64 rng(0x5eed);
    const uint32_t As[] = {1, 2, 3, 256, 1024, 4096, 65536};
    const uint32_t Ss[] = {32, 64, 128, 256};
    const uint32_t Cs[] = {1, 3, 32, 64};
    int i = 0;
    for (uint32_t A : As) {
        for (uint32_t L : {1u, 2u, 8u, 16u, 24u, 32u}) {
            const uint64_t n = (rng() % 3 == 0) ? rng() % 70 : 1000 + rng() % 20000;
            const double r = 0.1 + 0.85 * double(rng() % 1000) / 1000.0;
            round_trip(geometric_symbols(rng, n, A, r), A, L, Ss[i % 4], Cs[(i / 4) % 4]);
            ++i;
        }
    }
    // one used symbol, empty input
    round_trip(std::vector<uint16_t>(777, 5), 16, 4, 32, 2);
    round_trip(std::vector<uint16_t>(), 16, 4, 32, 2);
    // Fibonacci counts: the length limit binds
    {
        std::vector<uint64_t> h(30);
        h[0] = h[1] = 1;
        for (int s = 2; s < 30; ++s)
            h[s] = h[s - 1] + h[s - 2];
        std::vector<uint8_t> l1(30), l2(30);
        std::vector<uint32_t> c2(30);
        CHECK(hdref_code_lengths(h.data(), 30, 12, l1.data()) == 0);
        CHECK(hd_build_codebook(h.data(), 30, 12, l2.data(), c2.data()) == HD_OK);
        CHECK(l1 == l2);
        // counts near 2^40
        for (auto &v : h)
            v <<= 10;
        CHECK(hdref_code_lengths(h.data(), 30, 20, l1.data()) == 0);
        CHECK(hd_build_codebook(h.data(), 30, 20, l2.data(), c2.data()) == HD_OK);
        CHECK(l1 == l2);
        // infeasible: 30 used symbols, L = 4
        CHECK(hd_build_codebook(h.data(), 30, 4, l2.data(), c2.data()) == HD_ERR_INFEASIBLE);
        CHECK(hdref_code_lengths(h.data(), 30, 4, l1.data()) == -2);
    }
    // bad arguments
    {
        uint64_t h[4] = {1, 2, 3, 4};
        uint8_t l[4];
        uint32_t c[4];
        CHECK(hd_build_codebook(h, 0, 8, l, c) == HD_ERR_ARG);
        CHECK(hd_build_codebook(h, 4, 0, l, c) == HD_ERR_ARG);
        CHECK(hd_build_codebook(h, 4, 33, l, c) == HD_ERR_ARG);
        CHECK(hd_build_codebook(nullptr, 4, 8, l, c) == HD_ERR_ARG);
        hd_layout bad{48, 32};
        hd_stream_info si;
        const uint16_t x[3] = {0, 1, 2};
        CHECK(hd_build_codebook(h, 4, 8, l, c) == HD_OK);
        CHECK(hd_encode_ref(x, 3, l, c, 4, 8, &bad, nullptr, 0, nullptr, 0, nullptr, 0, &si) == HD_ERR_ARG);
        const uint16_t y[2] = {0, 9};
        hd_layout lay{32, 1};
        CHECK(hd_encode_ref(y, 2, l, c, 4, 8, &lay, nullptr, 0, nullptr, 0, nullptr, 0, &si) == HD_ERR_SYMBOL);
        CHECK(hd_stream_layout(10, 5, 4, 8, &lay, &si) == HD_ERR_CORRUPT);
        CHECK(std::strlen(hd_status_str(HD_ERR_CORRUPT)) > 0);
        CHECK(std::strlen(hd_status_str(static_cast<hd_status>(-99))) > 0);
    }
    std::printf("sanitized host checks: %d failures\n", g_fail);
    return g_fail ? 1 : 0;
}
