// SZ-style reconstruction after Huffman decoding, for gfx950.
//
// The decoded symbols are quantization codes of a 3-D field (Sec. II-A:
// error-bounded lossy compression; Sec. V-B-2 measures the whole cuSZ
// decompression around the decoder).  Each code is a first-order Lorenzo
// prediction residual of the prequantized integer field q, shifted by a
// radius, with code 0 marking a residual held in a separate outlier list
// (ascending flat index + true residual).  Reconstruction:
//
//   r(i,j,k) = code - radius, or the listed residual where code == 0;
//   q(i,j,k) = sum of r over the box [0,i] x [0,j] x [0,k]   (the inverse of
//              the predictor: an inclusive prefix sum along every axis);
//   x(i,j,k) = q * 2 eb, the float64 product converted to float32.
//
// Three kernels, all streaming HBM-bound work (no contraction, no MFMA):
//
//   k_lz_plane   one wavefront per block of R consecutive rows of one plane i.
//                Per row: codes -> residuals (outliers by binary search, only
//                for code-0 lanes), inclusive scan along k (8 per lane, DPP
//                across the wave, a scalar carry across 512-wide chunks), and
//                a running column sum over the block's rows kept in
//                registers.  The running sums -- the box sum over the block's
//                rows up to j and over k' <= k -- go to the output buffer as
//                int32; the block's column totals go to the carry table.
//                Rows of at most 512 values in whole 16-byte groups take
//                k_lz_plane_ring, which keeps the next rows' codes in flight.
//   k_lz_carry   one thread per (i, k): exclusive scan of the column totals
//                over the row blocks of plane i (in place), so each block gets
//                the sum over all rows above it.
//   k_lz_depth   one thread per column pair (j, k..k+1): walks i, adds the block carry
//                to the plane value, accumulates along i and overwrites the
//                int32 in the output buffer with the dequantized float32 (the
//                same element, read then written by the same thread).
//
// HBM bytes per element: 2 (codes) + 4 + 4 (int32 out, back in) + 4 (float
// out), plus 3 x 4 / R for the carry table.  1-D fields longer than 4096
// values (ni = nj = 1) take a reduce-then-scan over tiles instead: codes read
// twice, float32 written once (8 bytes per element).  Integer arithmetic is modulo
// 2^32: every q fits int32, so wrapped partial sums still end exact.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hd.h"
#include "hd_internal.h"

namespace {

constexpr uint32_t kLzBlock = 256;          // threads per workgroup, every kernel
constexpr uint32_t kLzChunk = 512;          // k values per wavefront pass (8 per lane)
constexpr uint32_t kLzMaxChunks = 8;        // rows up to 4096 values
constexpr uint32_t kLzDepthUnroll = 2;      // planes loaded ahead in k_lz_depth (measured best)
constexpr int kLzRing = 4;                  // rows in flight in k_lz_plane_ring
constexpr uint32_t kXcds = 8;               // accelerator complex dies of an MI355X
constexpr size_t kLzStatusBytes = 256;      // status word, padded

struct LzArgs {
    const uint16_t *codes;
    const uint64_t *oidx;
    const int32_t *oval;
    uint64_t n_out;
    uint32_t *status;
    uint32_t *out;        // int32 partials, then float32 values
    int32_t *q_out;       // optional
    uint32_t *carry;      // [ni][nb][nk]
    uint32_t ni, nj, nk, nb, rows;
    uint32_t radius;
    double two_eb;
};

// Inclusive sum over lanes 0..l of a wavefront (DPP row shifts within each
// 16-lane row, then the row broadcasts that carry across rows).
__device__ __forceinline__ uint32_t lz_wave_scan(uint32_t v)
{
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false));
    return v;
}

// The listed residual at flat index e (lower bound over the ascending index
// list).  Sets *miss when e is absent.
__device__ __forceinline__ uint32_t lz_outlier(const uint64_t *idx, const int32_t *val, uint64_t n, uint64_t e,
                                               bool *miss)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (idx[mid] < e)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < n && idx[lo] == e)
        return static_cast<uint32_t>(val[lo]);
    *miss = true;
    return 0;
}

constexpr uint32_t kLzPad = 0xffffffffu;     // a k past the row: no residual

// Codes of one lane's 8 consecutive k values starting at element e0 (k0 is
// the first one's k).  VEC: the 8 codes are one aligned 16-byte load.
template <bool VEC>
__device__ __forceinline__ void lz_load_codes(const LzArgs &a, uint64_t e0, uint32_t k0, uint32_t c[8])
{
    if (VEC) {
        if (k0 < a.nk) {
            const uint4 w = *reinterpret_cast<const uint4 *>(a.codes + e0);
            c[0] = w.x & 0xffffu; c[1] = w.x >> 16;
            c[2] = w.y & 0xffffu; c[3] = w.y >> 16;
            c[4] = w.z & 0xffffu; c[5] = w.z >> 16;
            c[6] = w.w & 0xffffu; c[7] = w.w >> 16;
        } else {
#pragma unroll
            for (int v = 0; v < 8; ++v)
                c[v] = kLzPad;
        }
    } else {
#pragma unroll
        for (int v = 0; v < 8; ++v)
            c[v] = (k0 + v < a.nk) ? a.codes[e0 + v] : kLzPad;
    }
}

template <bool VEC>
__device__ __forceinline__ void lz_store(const LzArgs &a, uint32_t *dst, uint64_t e0, uint32_t k0,
                                         const uint32_t s[8])
{
    if (VEC) {
        if (k0 < a.nk) {
            *reinterpret_cast<uint4 *>(dst + e0) = make_uint4(s[0], s[1], s[2], s[3]);
            *reinterpret_cast<uint4 *>(dst + e0 + 4) = make_uint4(s[4], s[5], s[6], s[7]);
        }
    } else {
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (k0 + v < a.nk)
                dst[e0 + v] = s[v];
    }
}

template <uint32_t NCH, bool VEC>
__global__ void __launch_bounds__(kLzBlock) k_lz_plane(LzArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t w = uint64_t(blockIdx.x) * (kLzBlock / 64) +
                       static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6)));
    if (w >= uint64_t(a.ni) * a.nb)
        return;
    const uint32_t i = static_cast<uint32_t>(w / a.nb);
    const uint32_t b = static_cast<uint32_t>(w - uint64_t(i) * a.nb);
    const uint32_t j0 = b * a.rows;
    const uint32_t j1 = min(a.nj, j0 + a.rows);

    uint32_t col[NCH][8];
#pragma unroll
    for (uint32_t c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < 8; ++v)
            col[c][v] = 0;

    bool miss = false;
    uint32_t cur[NCH][8];
    uint64_t row = (uint64_t(i) * a.nj + j0) * a.nk;
#pragma unroll
    for (uint32_t c = 0; c < NCH; ++c)
        lz_load_codes<VEC>(a, row + c * kLzChunk + lane * 8, c * kLzChunk + lane * 8, cur[c]);

    for (uint32_t j = j0; j < j1; ++j) {
        // the next row's codes are in flight while this row is scanned
        uint32_t nxt[NCH][8];
        const uint64_t nrow = row + a.nk;
        if (j + 1 < j1) {
#pragma unroll
            for (uint32_t c = 0; c < NCH; ++c)
                lz_load_codes<VEC>(a, nrow + c * kLzChunk + lane * 8, c * kLzChunk + lane * 8, nxt[c]);
        }
        uint32_t rowsum = 0;                 // wavefront-uniform carry along k
#pragma unroll
        for (uint32_t c = 0; c < NCH; ++c) {
            const uint32_t k0 = c * kLzChunk + lane * 8;
            const uint64_t e0 = row + k0;
            // residuals with code 0 taken as -radius first; each code-0
            // position then adds (listed residual + radius) to its suffix
            uint32_t s[8];
            uint32_t run = 0, zmask = 0;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const uint32_t code = cur[c][v];
                run += code == kLzPad ? 0u : code - a.radius;
                zmask |= code == 0 ? 1u << v : 0u;
                s[v] = run;
            }
            while (zmask) {
                const uint32_t v0 = static_cast<uint32_t>(__builtin_ctz(zmask));
                zmask &= zmask - 1;
                const uint32_t fix = lz_outlier(a.oidx, a.oval, a.n_out, e0 + v0, &miss) + a.radius;
#pragma unroll
                for (uint32_t v = 0; v < 8; ++v)
                    s[v] += v >= v0 ? fix : 0u;
                run += fix;
            }
            const uint32_t incl = lz_wave_scan(run);
            const uint32_t base = incl - run + rowsum;
            rowsum += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), 63));
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                col[c][v] += s[v] + base;
                s[v] = col[c][v];
            }
            lz_store<VEC>(a, a.out, e0, k0, s);
        }
        row = nrow;
        if (j + 1 < j1) {
#pragma unroll
            for (uint32_t c = 0; c < NCH; ++c)
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    cur[c][v] = nxt[c][v];
        }
    }
    if (a.nb > 1) {
        const uint64_t t0 = (uint64_t(i) * a.nb + b) * a.nk;
#pragma unroll
        for (uint32_t c = 0; c < NCH; ++c) {
            const uint32_t k0 = c * kLzChunk + lane * 8;
            lz_store<VEC>(a, a.carry, t0 + k0, k0, col[c]);
        }
    }
    if (miss)
        atomicOr(a.status, hd::kErrNoOutlier);
}

// Rows of at most 512 values in whole 16-byte groups: each lane owns 8
// consecutive k for the whole block, and the codes of the next PD rows are in
// flight (a ring of packed 16-byte loads) while a row is scanned.
template <int PD>
__global__ void __launch_bounds__(kLzBlock) k_lz_plane_ring(LzArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t w = uint64_t(blockIdx.x) * (kLzBlock / 64) +
                       static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6)));
    if (w >= uint64_t(a.ni) * a.nb)
        return;
    const uint32_t i = static_cast<uint32_t>(w / a.nb);
    const uint32_t b = static_cast<uint32_t>(w - uint64_t(i) * a.nb);
    const uint32_t j0 = b * a.rows;
    const uint32_t j1 = min(a.nj, j0 + a.rows);
    const uint32_t k0 = lane * 8;
    const bool act = k0 < a.nk;
    const uint64_t base_e = (uint64_t(i) * a.nj + j0) * a.nk + k0;

    uint32_t col[8];
#pragma unroll
    for (int v = 0; v < 8; ++v)
        col[v] = 0;
    bool miss = false;
    uint4 buf[PD];
#pragma unroll
    for (int d = 0; d < PD; ++d)
        buf[d] = (act && j0 + d < j1) ? *reinterpret_cast<const uint4 *>(a.codes + base_e + uint64_t(d) * a.nk)
                                      : make_uint4(0, 0, 0, 0);
    for (uint32_t j = j0; j < j1; j += PD) {
#pragma unroll
        for (int d = 0; d < PD; ++d) {
            if (j + d < j1) {
                const uint4 wv = buf[d];
                const uint64_t e0 = base_e + uint64_t(j + d - j0) * a.nk;
                if (act && j + d + PD < j1)
                    buf[d] = *reinterpret_cast<const uint4 *>(a.codes + e0 + uint64_t(PD) * a.nk);
                uint32_t c[8] = {wv.x & 0xffffu, wv.x >> 16, wv.y & 0xffffu, wv.y >> 16,
                                 wv.z & 0xffffu, wv.z >> 16, wv.w & 0xffffu, wv.w >> 16};
                uint32_t s[8];
                uint32_t run = 0, zmask = 0;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    run += act ? c[v] - a.radius : 0u;
                    zmask |= (act && c[v] == 0) ? 1u << v : 0u;
                    s[v] = run;
                }
                while (zmask) {
                    const uint32_t v0 = static_cast<uint32_t>(__builtin_ctz(zmask));
                    zmask &= zmask - 1;
                    const uint32_t fix = lz_outlier(a.oidx, a.oval, a.n_out, e0 + v0, &miss) + a.radius;
#pragma unroll
                    for (uint32_t v = 0; v < 8; ++v)
                        s[v] += v >= v0 ? fix : 0u;
                    run += fix;
                }
                const uint32_t incl = lz_wave_scan(run);
                const uint32_t base = incl - run;
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    col[v] += s[v] + base;
                if (act) {
                    *reinterpret_cast<uint4 *>(a.out + e0) = make_uint4(col[0], col[1], col[2], col[3]);
                    *reinterpret_cast<uint4 *>(a.out + e0 + 4) = make_uint4(col[4], col[5], col[6], col[7]);
                }
            }
        }
    }
    if (a.nb > 1 && act) {
        uint32_t *t = a.carry + (uint64_t(i) * a.nb + b) * a.nk + k0;
        *reinterpret_cast<uint4 *>(t) = make_uint4(col[0], col[1], col[2], col[3]);
        *reinterpret_cast<uint4 *>(t + 4) = make_uint4(col[4], col[5], col[6], col[7]);
    }
    if (miss)
        atomicOr(a.status, hd::kErrNoOutlier);
}

// Exclusive scan over row blocks of each plane's column totals (in place).
__global__ void __launch_bounds__(kLzBlock) k_lz_carry(LzArgs a)
{
    const uint64_t t = uint64_t(blockIdx.x) * kLzBlock + threadIdx.x;
    if (t >= uint64_t(a.ni) * a.nk)
        return;
    const uint32_t i = static_cast<uint32_t>(t / a.nk);   // t < 2^32 * 4096
    const uint32_t k = static_cast<uint32_t>(t - uint64_t(i) * a.nk);
    uint32_t *p = a.carry + uint64_t(i) * a.nb * a.nk + k;
    uint32_t acc = 0;
    for (uint32_t b = 0; b < a.nb; ++b) {
        const uint32_t v = p[uint64_t(b) * a.nk];
        p[uint64_t(b) * a.nk] = acc;
        acc += v;
    }
}

template <int N> struct LzVec;
template <> struct LzVec<1> { using T = uint32_t; };
template <> struct LzVec<2> { using T = uint2; };
__device__ __forceinline__ uint32_t &lz_el(uint32_t &v, int) { return v; }
__device__ __forceinline__ uint32_t &lz_el(uint2 &v, int c) { return c ? v.y : v.x; }

// COLS adjacent columns per thread (COLS = 2 needs an even nk: a pair never
// straddles two rows).  Planes are loaded kLzDepthUnroll at a time; the
// final values are written with non-temporal stores (nothing reads them here).
template <bool CARRY, bool QOUT, int COLS>
__global__ void __launch_bounds__(kLzBlock) k_lz_depth(LzArgs a)
{
    using V = typename LzVec<COLS>::T;
    // Workgroups are dealt to the 8 XCDs round robin; renumber them so that
    // consecutive rows (which read the same carry-table lines) share one
    // XCD's L2 instead of fetching each line once per XCD.
    uint32_t g = blockIdx.x;
    if (gridDim.x % kXcds == 0)
        g = (g % kXcds) * (gridDim.x / kXcds) + g / kXcds;
    const uint64_t t = (uint64_t(g) * kLzBlock + threadIdx.x) * COLS;
    const uint64_t plane = uint64_t(a.nj) * a.nk;
    if (t >= plane)
        return;
    uint32_t j;
    if (plane <= 0xffffffffu)
        j = static_cast<uint32_t>(t) / a.nk;
    else
        j = static_cast<uint32_t>(t / a.nk);
    const uint32_t k = static_cast<uint32_t>(t - uint64_t(j) * a.nk);
    const uint64_t cstride = uint64_t(a.nb) * a.nk;
    const uint32_t *cp = a.carry + uint64_t(j / a.rows) * a.nk + k;
    uint32_t acc[COLS];
#pragma unroll
    for (int c = 0; c < COLS; ++c)
        acc[c] = 0;
    for (uint32_t i0 = 0; i0 < a.ni; i0 += kLzDepthUnroll) {
        V v[kLzDepthUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kLzDepthUnroll; ++u) {
            if (i0 + u < a.ni) {
                v[u] = *reinterpret_cast<const V *>(a.out + uint64_t(i0 + u) * plane + t);
                if (CARRY) {
                    V cv = *reinterpret_cast<const V *>(cp + uint64_t(i0 + u) * cstride);
#pragma unroll
                    for (int c = 0; c < COLS; ++c)
                        lz_el(v[u], c) += lz_el(cv, c);
                }
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kLzDepthUnroll; ++u) {
            if (i0 + u < a.ni) {
                const uint64_t e = uint64_t(i0 + u) * plane + t;
#pragma unroll
                for (int c = 0; c < COLS; ++c) {
                    acc[c] += lz_el(v[u], c);
                    const double x = static_cast<double>(static_cast<int32_t>(acc[c])) * a.two_eb;
                    __builtin_nontemporal_store(__float_as_uint(static_cast<float>(x)), a.out + e + c);
                    if (QOUT)
                        __builtin_nontemporal_store(static_cast<int32_t>(acc[c]), a.q_out + e + c);
                }
            }
        }
    }
}

// ---- long 1-D fields (ni = nj = 1, nk > 4096): q is a plain prefix sum of
// the residuals, done as reduce-then-scan over tiles of 4096 values.

constexpr uint32_t kLzTile = kLzBlock * 16;    // values per tile (16 per thread)

// Residuals of the thread's 16 values starting at element e0 (< n), as
// inclusive running sums in s[]; returns the thread's total.
__device__ __forceinline__ uint32_t lz_line_run(const LzArgs &a, uint64_t n, uint64_t e0, bool vec, uint32_t s[16],
                                                bool *miss)
{
    uint32_t c[16];
    if (vec && e0 + 16 <= n) {
        const uint4 u = *reinterpret_cast<const uint4 *>(a.codes + e0);
        const uint4 v = *reinterpret_cast<const uint4 *>(a.codes + e0 + 8);
        const uint32_t w[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            c[2 * q] = w[q] & 0xffffu;
            c[2 * q + 1] = w[q] >> 16;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            c[q] = e0 + q < n ? a.codes[e0 + q] : kLzPad;
    }
    uint32_t run = 0, zmask = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        run += c[q] == kLzPad ? 0u : c[q] - a.radius;
        zmask |= c[q] == 0 ? 1u << q : 0u;
        s[q] = run;
    }
    while (zmask) {
        const uint32_t q0 = static_cast<uint32_t>(__builtin_ctz(zmask));
        zmask &= zmask - 1;
        const uint32_t fix = lz_outlier(a.oidx, a.oval, a.n_out, e0 + q0, miss) + a.radius;
#pragma unroll
        for (uint32_t q = 0; q < 16; ++q)
            s[q] += q >= q0 ? fix : 0u;
        run += fix;
    }
    return run;
}

// Exclusive prefix of v over the 256 threads of the workgroup; *all = total.
__device__ __forceinline__ uint32_t lz_block_excl(uint32_t v, uint32_t *lds4, uint32_t *all)
{
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t incl = lz_wave_scan(v);
    if (lane == 63)
        lds4[wv] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < kLzBlock / 64; ++w) {
        before += w < wv ? lds4[w] : 0u;
        tot += lds4[w];
    }
    *all = tot;
    return before + incl - v;
}

__global__ void __launch_bounds__(kLzBlock) k_lz_line_sum(LzArgs a, uint32_t *tile_sum, bool vec)
{
    __shared__ uint32_t lds4[kLzBlock / 64];
    const uint64_t n = a.nk;
    const uint64_t e0 = uint64_t(blockIdx.x) * kLzTile + uint64_t(threadIdx.x) * 16;
    bool miss = false;
    uint32_t s[16];
    const uint32_t t = lz_line_run(a, n, e0, vec, s, &miss);
    uint32_t all;
    lz_block_excl(t, lds4, &all);
    if (threadIdx.x == 0)
        tile_sum[blockIdx.x] = all;
    if (miss)
        atomicOr(a.status, hd::kErrNoOutlier);
}

// Tile sums -> exclusive tile offsets in two levels: each 1024-thread
// workgroup scans 1024 tile sums in place and leaves its total in group[g];
// then one workgroup scans the group totals in place (all modulo 2^32).
constexpr uint32_t kLzScanGroup = 1024;

__device__ __forceinline__ uint32_t lz_group_excl(uint32_t v, uint32_t *part, uint32_t *all)
{
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t incl = lz_wave_scan(v);
    if (lane == 63)
        part[wv] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t w = 0; w < kLzScanGroup / 64; ++w) {
        before += w < wv ? part[w] : 0u;
        tot += part[w];
    }
    *all = tot;
    return before + incl - v;
}

__global__ void __launch_bounds__(kLzScanGroup) k_lz_line_scan(uint32_t *tile_sum, uint32_t nt, uint32_t *group)
{
    __shared__ uint32_t part[kLzScanGroup / 64];
    const uint32_t b = blockIdx.x * kLzScanGroup + threadIdx.x;
    const uint32_t v = b < nt ? tile_sum[b] : 0u;
    uint32_t all;
    const uint32_t ex = lz_group_excl(v, part, &all);
    if (b < nt)
        tile_sum[b] = ex;
    if (threadIdx.x == 0)
        group[blockIdx.x] = all;
}

__global__ void __launch_bounds__(kLzScanGroup) k_lz_line_top(uint32_t *group, uint32_t ng)
{
    __shared__ uint32_t part[kLzScanGroup / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < ng; base += kLzScanGroup) {
        const uint32_t b = base + threadIdx.x;
        const uint32_t v = b < ng ? group[b] : 0u;
        uint32_t all;
        const uint32_t ex = lz_group_excl(v, part, &all);
        if (b < ng)
            group[b] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0)
            carry += all;
        __syncthreads();
    }
}

template <bool QOUT>
__global__ void __launch_bounds__(kLzBlock) k_lz_line_out(LzArgs a, const uint32_t *tile_off, const uint32_t *group,
                                                           bool vec, bool ovec)
{
    __shared__ uint32_t lds4[kLzBlock / 64];
    const uint64_t n = a.nk;
    const uint64_t e0 = uint64_t(blockIdx.x) * kLzTile + uint64_t(threadIdx.x) * 16;
    bool miss = false;
    uint32_t s[16];
    const uint32_t t = lz_line_run(a, n, e0, vec, s, &miss);
    uint32_t all;
    const uint32_t base = lz_block_excl(t, lds4, &all) + tile_off[blockIdx.x] + group[blockIdx.x / kLzScanGroup];
    uint32_t f[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        s[q] += base;
        const double x = static_cast<double>(static_cast<int32_t>(s[q])) * a.two_eb;
        f[q] = __float_as_uint(static_cast<float>(x));
    }
    // a thread's 16 values are 64 contiguous bytes: whole 16-byte stores, so
    // every line is written in full
    if (ovec && e0 + 16 <= n) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            *reinterpret_cast<uint4 *>(a.out + e0 + 4 * g) = make_uint4(f[4 * g], f[4 * g + 1], f[4 * g + 2], f[4 * g + 3]);
            if (QOUT)
                *reinterpret_cast<uint4 *>(a.q_out + e0 + 4 * g) =
                    make_uint4(s[4 * g], s[4 * g + 1], s[4 * g + 2], s[4 * g + 3]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (e0 + q < n) {
                a.out[e0 + q] = f[q];
                if (QOUT)
                    a.q_out[e0 + q] = static_cast<int32_t>(s[q]);
            }
        }
    }
    if (miss)
        atomicOr(a.status, hd::kErrNoOutlier);
}

// Clears the status word and the word after it (the count of decode status
// slots, which hd_decode_status_bits reads; none here).
__global__ void k_lz_clear(uint32_t *status)
{
    if (threadIdx.x == 0) {
        status[0] = 0;
        status[1] = 0;
    }
}

// Rows per wavefront block: 32, halved (down to 8) while the plane kernel
// would have fewer than 4096 wavefronts.
uint32_t lz_rows(uint32_t ni, uint32_t nj)
{
    uint32_t r = 32;
    while (r > 8 && uint64_t(ni) * ((uint64_t(nj) + r - 1) / r) < 4096)
        r >>= 1;
    return r;
}

bool lz_line(uint32_t ni, uint32_t nj, uint32_t nk)
{
    return ni == 1 && nj == 1 && nk > kLzChunk * kLzMaxChunks;
}

size_t lz_ws_bytes(uint32_t ni, uint32_t nj, uint32_t nk)
{
    if (lz_line(ni, nj, nk)) {
        const uint64_t nt = (uint64_t(nk) + kLzTile - 1) / kLzTile;
        return kLzStatusBytes + nt * 4 + (nt + kLzScanGroup - 1) / kLzScanGroup * 4;
    }
    const uint32_t r = lz_rows(ni, nj);
    const uint64_t nb = (uint64_t(nj) + r - 1) / r;
    return kLzStatusBytes + (nb > 1 ? size_t(ni) * nb * nk * 4 : 0);
}

using PlaneKernel = void (*)(LzArgs);

template <bool VEC>
PlaneKernel plane_kernel(uint32_t nch)
{
    switch (nch) {
    case 1: return k_lz_plane<1, VEC>;
    case 2: return k_lz_plane<2, VEC>;
    case 3:
    case 4: return k_lz_plane<4, VEC>;
    default: return k_lz_plane<8, VEC>;
    }
}

template <int COLS>
PlaneKernel depth_kernel(bool carry, bool qout)
{
    return carry ? (qout ? k_lz_depth<true, true, COLS> : k_lz_depth<true, false, COLS>)
                 : (qout ? k_lz_depth<false, true, COLS> : k_lz_depth<false, false, COLS>);
}

}  // namespace

extern "C" size_t hd_lorenzo_workspace_size(uint32_t ni, uint32_t nj, uint32_t nk)
{
    return lz_ws_bytes(ni, nj, nk);
}

extern "C" hd_status hd_lorenzo_reconstruct(const uint16_t *codes, uint32_t ni, uint32_t nj, uint32_t nk,
                                            uint32_t radius, const uint64_t *outlier_idx,
                                            const int32_t *outlier_val, uint64_t n_outliers, double eb,
                                            float *out, int32_t *q_out, void *workspace, size_t ws_bytes,
                                            void *hip_stream)
{
    const uint64_t n = uint64_t(ni) * nj * nk;
    if (!workspace || ws_bytes < lz_ws_bytes(ni, nj, nk) || radius == 0 || !(eb > 0.0) || !std::isfinite(eb))
        return HD_ERR_ARG;
    if (n > 0 && (!codes || !out))
        return HD_ERR_ARG;
    if (n_outliers > 0 && (!outlier_idx || !outlier_val))
        return HD_ERR_ARG;
    if (nk > kLzChunk * kLzMaxChunks && !lz_line(ni, nj, nk))
        return HD_ERR_UNSUPPORTED;
    if (reinterpret_cast<uintptr_t>(workspace) % 16)
        return HD_ERR_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    uint32_t *status = static_cast<uint32_t *>(workspace);
    hipLaunchKernelGGL(k_lz_clear, dim3(1), dim3(64), 0, stream, status);
    if (hipGetLastError() != hipSuccess)
        return HD_ERR_DEVICE;
    if (n == 0)
        return HD_OK;

    LzArgs a{};
    a.codes = codes;
    a.oidx = outlier_idx;
    a.oval = outlier_val;
    a.n_out = n_outliers;
    a.status = status;
    a.out = reinterpret_cast<uint32_t *>(out);
    a.q_out = q_out;
    a.rows = lz_rows(ni, nj);
    a.nb = (nj + a.rows - 1) / a.rows;
    a.carry = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + kLzStatusBytes);
    a.ni = ni;
    a.nj = nj;
    a.nk = nk;
    a.radius = radius;
    a.two_eb = 2.0 * eb;

    if (lz_line(ni, nj, nk)) {
        uint32_t *tiles = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + kLzStatusBytes);
        const uint32_t nt = static_cast<uint32_t>((uint64_t(nk) + kLzTile - 1) / kLzTile);
        const bool lvec = reinterpret_cast<uintptr_t>(codes) % 16 == 0;
        const bool ovec = reinterpret_cast<uintptr_t>(out) % 16 == 0 && reinterpret_cast<uintptr_t>(q_out) % 16 == 0;
        const uint32_t ng = (nt + kLzScanGroup - 1) / kLzScanGroup;
        uint32_t *groups = tiles + nt;
        hipLaunchKernelGGL(k_lz_line_sum, dim3(nt), dim3(kLzBlock), 0, stream, a, tiles, lvec);
        hipLaunchKernelGGL(k_lz_line_scan, dim3(ng), dim3(kLzScanGroup), 0, stream, tiles, nt, groups);
        hipLaunchKernelGGL(k_lz_line_top, dim3(1), dim3(kLzScanGroup), 0, stream, groups, ng);
        if (q_out)
            hipLaunchKernelGGL(k_lz_line_out<true>, dim3(nt), dim3(kLzBlock), 0, stream, a, tiles, groups, lvec, ovec);
        else
            hipLaunchKernelGGL(k_lz_line_out<false>, dim3(nt), dim3(kLzBlock), 0, stream, a, tiles, groups, lvec,
                               ovec);
        return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
    }
    const bool vec = nk % 8 == 0 && reinterpret_cast<uintptr_t>(codes) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(out) % 16 == 0;
    const uint32_t nch = (nk + kLzChunk - 1) / kLzChunk;
    const uint64_t waves = uint64_t(ni) * a.nb;
    const uint64_t g1 = (waves + kLzBlock / 64 - 1) / (kLzBlock / 64);
    const uint64_t g2 = (uint64_t(ni) * nk + kLzBlock - 1) / kLzBlock;
    if (g1 > 0x7fffffffu || g2 > 0x7fffffffu || (uint64_t(nj) * nk + kLzBlock - 1) / kLzBlock > 0x7fffffffu)
        return HD_ERR_UNSUPPORTED;

    PlaneKernel plane = vec && nch == 1 ? k_lz_plane_ring<kLzRing>
                                        : vec ? plane_kernel<true>(nch) : plane_kernel<false>(nch);
    hipLaunchKernelGGL(plane, dim3(uint32_t(g1)), dim3(kLzBlock), 0, stream, a);
    if (a.nb > 1)
        hipLaunchKernelGGL(k_lz_carry, dim3(uint32_t(g2)), dim3(kLzBlock), 0, stream, a);
    const bool pairs = nk % 2 == 0 && reinterpret_cast<uintptr_t>(out) % 8 == 0 &&
                       reinterpret_cast<uintptr_t>(q_out) % 8 == 0;
    PlaneKernel depth = pairs ? depth_kernel<2>(a.nb > 1, q_out != nullptr)
                              : depth_kernel<1>(a.nb > 1, q_out != nullptr);
    const uint64_t g3 = (uint64_t(nj) * nk / (pairs ? 2 : 1) + kLzBlock - 1) / kLzBlock;
    hipLaunchKernelGGL(depth, dim3(uint32_t(g3)), dim3(kLzBlock), 0, stream, a);
    return hipGetLastError() == hipSuccess ? HD_OK : HD_ERR_DEVICE;
}
