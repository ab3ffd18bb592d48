// Huffman encoding on the device, for gfx950: the compress side of the
// stream format read by the decoders (Sec. II-B codewords, Sec. III-B 32-bit
// units, Sec. III-C gap array, chunk offsets).
//
//   k_enc_hist   histogram of the symbols: a persistent grid, counts in LDS
//                per workgroup over many blocks, then one 64-bit atomic add
//                per used bin and workgroup.
//   k_enc_plan   per block of 4096 symbols, the sum of their code lengths;
//                flags symbols without a codeword.  (Plan and write stage the
//                codebook in LDS for alphabets up to 16384.)
//   k_enc_scan   one workgroup: exclusive scan of the block sums (64-bit
//                bit offsets) and the stream's total bits.
//   k_enc_write  per block: each thread takes 16 consecutive symbols, finds
//                its first bit by a workgroup scan over the block, and packs
//                its codewords MSB first into 32-bit units of an LDS stage
//                (a unit shared with a neighbour thread is OR-ed there); the
//                block then stores its units coalesced, with an atomic OR
//                only on its first and last unit, which it may share with
//                the neighbour blocks (units start zeroed).  A
//                symbol whose codeword ends at or past a subsequence boundary
//                k*S (and starts before it) writes gap[k]; a symbol after
//                which a chunk boundary falls records its index + 1 as that
//                chunk's offset (the output index of its first codeword).
//
// HBM bytes per symbol: 2 (plan) + 2 (write) + the bitstream (zero fill, then
// written) + one gap byte per subsequence and 8 B per chunk.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hd.h"
#include "hd_internal.h"

namespace {

constexpr uint32_t kEncBlock = 256;                    // threads per workgroup
constexpr uint32_t kEncPer = 16;                       // symbols per thread
constexpr uint64_t kEncSyms = kEncBlock * kEncPer;     // symbols per block
constexpr uint32_t kHistLdsBins = 16384;               // LDS histogram up to this alphabet
constexpr uint32_t kHistGroups = 1024;                 // persistent workgroups of the histogram
constexpr uint32_t kStageWords = kEncSyms + 2;         // a block's units: <= 4096 x 32 bits, +1 partial
constexpr size_t kEncHead = 256;                       // status word + total bits
constexpr uint32_t kTabLdsSyms = 16384;                // codebook in LDS up to this alphabet

struct EncWs {
    uint32_t *status;      // byte 0 (byte 4: zero, no decode status slots)
    uint64_t *total;       // byte 8
    uint32_t *block_bits;  // [nblk]
    uint64_t *block_off;   // [nblk]
};

size_t enc_ws_bytes(uint64_t n)
{
    const uint64_t nblk = (n + kEncSyms - 1) / kEncSyms;
    return kEncHead + ((nblk * 4 + 15) & ~uint64_t(15)) + nblk * 8;
}

EncWs enc_ws(void *ws, uint64_t n)
{
    const uint64_t nblk = (n + kEncSyms - 1) / kEncSyms;
    char *p = static_cast<char *>(ws);
    EncWs w;
    w.status = reinterpret_cast<uint32_t *>(p);
    w.total = reinterpret_cast<uint64_t *>(p + 8);
    w.block_bits = reinterpret_cast<uint32_t *>(p + kEncHead);
    w.block_off = reinterpret_cast<uint64_t *>(p + kEncHead + ((nblk * 4 + 15) & ~uint64_t(15)));
    return w;
}

__device__ __forceinline__ uint32_t enc_wave_scan(uint32_t v)
{
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false));
    return v;
}

// Exclusive scan of one value per thread over a 256-thread workgroup; also
// returns the workgroup total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds4, uint32_t *total)
{
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t incl = enc_wave_scan(v);
    if (lane == 63)
        lds4[wv] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (uint32_t w = 0; w < kEncBlock / 64; ++w) {
        const uint32_t s = lds4[w];
        before += w < wv ? s : 0u;
        all += s;
    }
    *total = all;
    return before + incl - v;
}

// The thread's 16 symbols (a partial block's tail reads nothing past n).
__device__ __forceinline__ void load_syms(const uint16_t *syms, uint64_t n, uint64_t s0, uint32_t x[kEncPer],
                                          bool vec)
{
    if (vec && s0 + kEncPer <= n) {
        const uint4 a = *reinterpret_cast<const uint4 *>(syms + s0);
        const uint4 b = *reinterpret_cast<const uint4 *>(syms + s0 + 8);
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            x[2 * q] = w[q] & 0xffffu;
            x[2 * q + 1] = w[q] >> 16;
        }
    } else {
#pragma unroll
        for (uint32_t q = 0; q < kEncPer; ++q)
            x[q] = s0 + q < n ? syms[s0 + q] : 0xffffffffu;
    }
}

// A persistent grid: each workgroup counts many blocks of symbols into one
// LDS histogram and adds it to the global one once, so the global 64-bit
// atomics (which contend on the few hot bins of a peaked distribution) number
// workgroups x used bins rather than blocks x used bins.  Alphabets beyond
// the LDS size count with global atomics directly.
__global__ void __launch_bounds__(kEncBlock) k_enc_hist(const uint16_t *syms, uint64_t n, uint32_t A,
                                                        unsigned long long *hist, bool vec)
{
    __shared__ uint32_t h[kHistLdsBins];
    const bool lds = A <= kHistLdsBins;
    if (lds) {
        for (uint32_t b = threadIdx.x; b < A; b += kEncBlock)
            h[b] = 0;
        __syncthreads();
    }
    const uint64_t nblk = (n + kEncSyms - 1) / kEncSyms;
    for (uint64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const uint64_t s0 = blk * kEncSyms + uint64_t(threadIdx.x) * kEncPer;
        uint32_t x[kEncPer];
        load_syms(syms, n, s0, x, vec);
#pragma unroll
        for (uint32_t q = 0; q < kEncPer; ++q) {
            if (x[q] < A) {
                if (lds)
                    atomicAdd(&h[x[q]], 1u);
                else
                    atomicAdd(&hist[x[q]], 1ull);
            }
        }
    }
    if (lds) {
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < A; b += kEncBlock)
            if (h[b])
                atomicAdd(&hist[b], static_cast<unsigned long long>(h[b]));
    }
}

__global__ void __launch_bounds__(kEncBlock) k_enc_plan(const uint16_t *syms, uint64_t n, const uint8_t *len,
                                                        uint32_t A, uint32_t *block_bits, uint32_t *status, bool vec)
{
    __shared__ uint32_t lds4[kEncBlock / 64];
    extern __shared__ uint32_t enc_dyn[];        // lengths (A bytes) when A <= kTabLdsSyms
    uint8_t *tl = reinterpret_cast<uint8_t *>(enc_dyn);
    const bool lds = A <= kTabLdsSyms;
    if (lds) {
        for (uint32_t b = threadIdx.x; b < A; b += kEncBlock)
            tl[b] = len[b];
        __syncthreads();
    }
    const uint64_t s0 = uint64_t(blockIdx.x) * kEncSyms + uint64_t(threadIdx.x) * kEncPer;
    uint32_t x[kEncPer];
    load_syms(syms, n, s0, x, vec);
    uint32_t bits = 0;
    bool bad = false;
#pragma unroll
    for (uint32_t q = 0; q < kEncPer; ++q) {
        if (x[q] == 0xffffffffu)
            continue;
        const uint32_t l = x[q] < A ? (lds ? tl[x[q]] : len[x[q]]) : 0u;
        bad |= l == 0;
        bits += l;
    }
    uint32_t total;
    block_excl_scan(bits, lds4, &total);
    if (threadIdx.x == 0)
        block_bits[blockIdx.x] = total;
    if (bad)
        atomicOr(status, hd::kErrBadCode);
}

// One workgroup: block_off = exclusive scan of block_bits; *total = the sum.
__global__ void __launch_bounds__(1024) k_enc_scan(const uint32_t *block_bits, uint64_t nblk, uint64_t *block_off,
                                                   uint64_t *total)
{
    __shared__ uint64_t part[1024 / 64];
    __shared__ uint64_t carry;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (uint64_t base = 0; base < nblk; base += 1024) {
        const uint64_t b = base + threadIdx.x;
        const uint32_t v = b < nblk ? block_bits[b] : 0u;
        // block sums are < 2^18, so a wave's inclusive sums fit 32 bits
        const uint32_t incl = enc_wave_scan(v);
        if (lane == 63)
            part[wv] = incl;
        __syncthreads();
        uint64_t before = carry, all = carry;
        for (uint32_t w = 0; w < 1024 / 64; ++w) {
            before += w < wv ? part[w] : 0u;
            all += part[w];
        }
        if (b < nblk)
            block_off[b] = before + (incl - v);
        __syncthreads();
        if (threadIdx.x == 0)
            carry = all;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *total = carry;
}

__global__ void k_enc_fill(uint32_t *p, uint64_t n)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0;
}

struct WriteArgs {
    const uint16_t *syms;
    uint64_t n;
    const uint8_t *len;
    const uint32_t *code;
    uint32_t A;
    uint32_t S;              // subsequence bits
    uint64_t CS;             // chunk bits = C * S
    uint32_t *words;
    uint64_t n_words;
    uint8_t *gap;
    uint64_t K;
    uint64_t *first;         // [M + 1] chunk offsets (the caller's array)
    uint64_t M;
    const uint64_t *block_off;
    const uint64_t *total;
    uint32_t *status;
    bool vec;
};

// A unit of the block's LDS stage: stored when this thread owns all of its
// 32 bits, else OR-ed (the stage starts zeroed).
__device__ __forceinline__ void put_stage(uint32_t *stage, uint32_t u, uint32_t v, bool whole)
{
    if (whole)
        stage[u] = v;
    else if (v)
        atomicOr(&stage[u], v);
}

__global__ void __launch_bounds__(kEncBlock) k_enc_write(WriteArgs a)
{
    __shared__ uint32_t lds4[kEncBlock / 64];
    __shared__ uint32_t stage[kStageWords];
    extern __shared__ uint32_t enc_dyn[];        // codes (A words), then lengths (A bytes)
    uint32_t *tc = enc_dyn;
    uint8_t *tl = reinterpret_cast<uint8_t *>(enc_dyn + a.A);
    const bool lds = a.A <= kTabLdsSyms;
    if (lds) {
        for (uint32_t b = threadIdx.x; b < a.A; b += kEncBlock) {
            tc[b] = a.code[b];
            tl[b] = a.len[b];
        }
        __syncthreads();
    }
    const uint64_t s0 = uint64_t(blockIdx.x) * kEncSyms + uint64_t(threadIdx.x) * kEncPer;
    uint32_t x[kEncPer];
    load_syms(a.syms, a.n, s0, x, a.vec);
    uint32_t l[kEncPer];
    uint32_t bits = 0;
#pragma unroll
    for (uint32_t q = 0; q < kEncPer; ++q) {
        l[q] = (x[q] < a.A) ? (lds ? tl[x[q]] : a.len[x[q]]) : 0u;
        bits += l[q];
    }
    uint32_t total;
    const uint32_t excl = block_excl_scan(bits, lds4, &total);
    const uint64_t start = a.block_off[blockIdx.x] + excl;
    const uint64_t n_bits = *a.total;
    bool oob = false;

    // the first subsequence and chunk boundaries after start; each codeword
    // (at most 32 bits <= S) passes at most one subsequence boundary
    uint64_t kb = start / a.S + 1;             // next subsequence index
    uint64_t kbit = kb * a.S;                  // its first bit
    uint64_t cb = start / a.CS + 1;            // next chunk index
    uint64_t cbit = cb * a.CS;

    // the block's units go to an LDS stage first: unit 0 of the stage is the
    // global unit holding the block's first bit
    const uint64_t bstart = a.block_off[blockIdx.x];
    const uint64_t u0 = bstart >> 5;
    for (uint32_t i = threadIdx.x; i < kStageWords; i += kEncBlock)
        stage[i] = 0;
    __syncthreads();

    // codewords, MSB first: acc holds np pending bits (low bits) that fill
    // unit w from its first bit; the thread's first unit begins with
    // start % 32 zero bits that belong to the previous thread
    uint64_t w = start >> 5;
    uint64_t acc = 0;
    uint32_t np = static_cast<uint32_t>(start & 31u);
    uint64_t s = start;
#pragma unroll
    for (uint32_t q = 0; q < kEncPer; ++q) {
        const uint32_t lq = l[q];
        if (lq == 0)
            continue;
        const uint32_t raw = lds ? tc[x[q]] : a.code[x[q]];
        const uint32_t c = raw & (lq == 32 ? 0xffffffffu : ((1u << lq) - 1u));
        acc = (acc << lq) | c;
        np += lq;
        if (np >= 32) {
            const uint32_t v = static_cast<uint32_t>(acc >> (np - 32));
            // whole unit of this thread when its first bit is not before start
            put_stage(stage, static_cast<uint32_t>(w - u0), v, (w << 5) >= start);
            ++w;
            np -= 32;
            acc &= np ? ((uint64_t(1) << np) - 1u) : 0u;
        }
        const uint64_t e = s + lq;
        // gap entry of the subsequence boundary inside (s, e]
        if (kbit <= e) {
            if (kb < a.K)
                a.gap[kb] = static_cast<uint8_t>(e - kbit);
            ++kb;
            kbit += a.S;
        }
        // chunks whose first codeword is the next one
        while (cbit <= e) {
            if (cb <= a.M)
                a.first[cb] = s0 + q + 1;
            ++cb;
            cbit += a.CS;
        }
        s = e;
    }
    if (np)
        put_stage(stage, static_cast<uint32_t>(w - u0), static_cast<uint32_t>(acc << (32 - np)), false);
    __syncthreads();

    // stage -> HBM: the block's first and last units may hold a neighbour
    // block's bits too (atomic OR), the ones between are the block's alone
    if (total) {
        const uint64_t bend = bstart + total;                 // one past the block's last bit
        const uint32_t nu = static_cast<uint32_t>(((bend + 31) >> 5) - u0);
        for (uint32_t i = threadIdx.x; i < nu; i += kEncBlock) {
            const uint64_t gw = u0 + i;
            if (gw >= a.n_words) {
                oob = true;
                continue;
            }
            const bool edge = (i == 0 && (bstart & 31u)) || (i == nu - 1 && (bend & 31u));
            if (edge)
                atomicOr(&a.words[gw], stage[i]);
            else
                a.words[gw] = stage[i];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (a.K)
            a.gap[0] = 0;
        a.first[0] = 0;
        // chunks that begin at or after the end of the stream
        for (uint64_t ch = (n_bits ? (n_bits - 1) / a.CS : 0) + 1; ch <= a.M; ++ch)
            if (n_bits == 0 || ch * a.CS >= n_bits)
                a.first[ch] = a.n;
    }
    if (oob)
        atomicOr(a.status, hd::kErrOutRange);
}

// Offsets of an empty stream: every chunk starts at output index 0.
__global__ void k_enc_zero_offsets(uint64_t *first, uint64_t M)
{
    for (uint64_t c = threadIdx.x; c <= M; c += blockDim.x)
        first[c] = 0;
}

// Clears the status word, the word after it (the count of decode status
// slots, which hd_decode_status_bits reads) and the planned total.
__global__ void k_enc_clear(uint32_t *status, uint64_t *total)
{
    if (threadIdx.x == 0) {
        status[0] = 0;
        status[1] = 0;
        *total = 0;
    }
}

uint32_t grid_of(uint64_t n, uint64_t per)
{
    return static_cast<uint32_t>((n + per - 1) / per);
}

}  // namespace

extern "C" size_t hd_encode_workspace_size(uint64_t n, uint32_t L, const hd_layout *lay)
{
    if (!lay || lay->subseq_bits == 0 || lay->chunk_subseqs == 0 || L == 0 || L > 32)
        return 0;
    // n * L bits bound the stream, hence the subsequence and chunk counts
    return enc_ws_bytes(n);
}

extern "C" hd_status hd_histogram(const uint16_t *syms, uint64_t n, uint32_t A, uint64_t *hist, void *hip_stream)
{
    if (!hist || A == 0 || A > 65536 || (n && !syms) || (n + kEncSyms - 1) / kEncSyms > 0x7fffffffu)
        return HD_ERR_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_enc_fill, dim3(grid_of(2 * uint64_t(A), 256)), dim3(256), 0, stream,
                       reinterpret_cast<uint32_t *>(hist), 2 * uint64_t(A));
    if (n) {
        const bool vec = reinterpret_cast<uintptr_t>(syms) % 16 == 0;
        const uint32_t g = grid_of(n, kEncSyms) < kHistGroups ? grid_of(n, kEncSyms) : kHistGroups;
        hipLaunchKernelGGL(k_enc_hist, dim3(g), dim3(kEncBlock), 0, stream, syms, n, A,
                           reinterpret_cast<unsigned long long *>(hist), vec);
    }
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}

extern "C" hd_status hd_encode_plan(const uint16_t *syms, uint64_t n, const uint8_t *lengths, uint32_t A,
                                    void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!workspace || ws_bytes < enc_ws_bytes(n) || !lengths || A == 0 || A > 65536 || (n && !syms) ||
        reinterpret_cast<uintptr_t>(workspace) % 16 || (n + kEncSyms - 1) / kEncSyms > 0x7fffffffu)
        return HD_ERR_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const EncWs w = enc_ws(workspace, n);
    const uint64_t nblk = (n + kEncSyms - 1) / kEncSyms;
    hipLaunchKernelGGL(k_enc_clear, dim3(1), dim3(64), 0, stream, w.status, w.total);
    if (n) {
        const bool vec = reinterpret_cast<uintptr_t>(syms) % 16 == 0;
        const size_t lds = A <= kTabLdsSyms ? A : 0;
        hipLaunchKernelGGL(k_enc_plan, dim3(static_cast<uint32_t>(nblk)), dim3(kEncBlock), lds, stream, syms, n,
                           lengths, A, w.block_bits, w.status, vec);
        hipLaunchKernelGGL(k_enc_scan, dim3(1), dim3(1024), 0, stream, w.block_bits, nblk, w.block_off, w.total);
    }
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}

extern "C" hd_status hd_encode_bits(const void *workspace, uint64_t *n_bits, void *hip_stream)
{
    if (!workspace || !n_bits)
        return HD_ERR_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return HD_ERR_DEVICE;
    uint64_t head[2] = {0, 0};
    if (hipMemcpy(head, workspace, sizeof(head), hipMemcpyDeviceToHost) != hipSuccess)
        return HD_ERR_DEVICE;
    *n_bits = head[1];
    return (head[0] & 0xffffffffu) ? HD_ERR_SYMBOL : HD_OK;
}

extern "C" hd_status hd_encode_write(const uint16_t *syms, uint64_t n, const uint8_t *lengths, const uint32_t *codes,
                                     uint32_t A, const hd_layout *lay, uint32_t *words, uint64_t n_words,
                                     uint8_t *gap, uint64_t n_subseq, uint64_t *chunk_offsets, uint64_t n_chunks,
                                     void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!lay || lay->subseq_bits == 0 || lay->subseq_bits % 32 || lay->chunk_subseqs == 0)
        return HD_ERR_ARG;
    if (!workspace || ws_bytes < enc_ws_bytes(n) || !lengths || !codes || A == 0 ||
        A > 65536 || (n && !syms) || !words || n_words < 2 || (n_subseq && !gap) || !chunk_offsets ||
        reinterpret_cast<uintptr_t>(workspace) % 16 || n_chunks != (n_subseq + lay->chunk_subseqs - 1) /
        lay->chunk_subseqs)
        return HD_ERR_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const EncWs w = enc_ws(workspace, n);
    const uint64_t nblk = (n + kEncSyms - 1) / kEncSyms;
    hipLaunchKernelGGL(k_enc_fill, dim3(grid_of(n_words, 256 * 16)), dim3(256), 0, stream, words, n_words);
    if (n) {
        WriteArgs a{};
        a.syms = syms;
        a.n = n;
        a.len = lengths;
        a.code = codes;
        a.A = A;
        a.S = lay->subseq_bits;
        a.CS = uint64_t(lay->subseq_bits) * lay->chunk_subseqs;
        a.words = words;
        a.n_words = n_words;
        a.gap = gap;
        a.K = n_subseq;
        a.first = chunk_offsets;
        a.M = n_chunks;
        a.block_off = w.block_off;
        a.total = w.total;
        a.status = w.status;
        a.vec = reinterpret_cast<uintptr_t>(syms) % 16 == 0;
        const size_t lds = A <= kTabLdsSyms ? size_t(A) * 5 : 0;
        hipLaunchKernelGGL(k_enc_write, dim3(static_cast<uint32_t>(nblk)), dim3(kEncBlock), lds, stream, a);
    } else {
        hipLaunchKernelGGL(k_enc_zero_offsets, dim3(1), dim3(64), 0, stream, chunk_offsets, n_chunks);
    }
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}
