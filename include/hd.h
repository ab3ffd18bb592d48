/*
 * hd.h -- canonical-Huffman decoding of uint16 quantization-code streams on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is the lossless stage of SZ-style error-bounded lossy
 * decompression: quantization codes (fixed-length uint16 input symbols) were
 * Huffman-coded into variable-length prefix-free codewords (paper Sec. II-B,
 * adapted to multi-byte symbols in Sec. IV); decoding turns the codeword
 * bitstream back into the uint16 array, whose byte size defines throughput
 * (Table II caption: GB/s relative to the quantization codes).  Decoding stays
 * on the device with no host transfer (Sec. I, in-memory use case).
 *
 * Stream format (all integers native little-endian):
 *   words        uint32[n_words], the bitstream in 32-bit units (Sec. III-B);
 *                stream bit i is bit (31 - i%32) of words[i/32] (MSB first);
 *                codewords are written MSB first; bits past n_bits are 0;
 *                n_words = n_subseq * subseq_bits / 32 + 2 (two zero guard
 *                units so a 64-bit window at any bit < n_bits stays inside).
 *   gap          uint8[n_subseq] (Sec. III-C, the gap array, one byte per
 *                subsequence): gap[k] = p_k - k*S, p_k the first codeword
 *                start at or after bit k*S, the stream end counting as a
 *                start.  Always 0 <= gap[k] < max_len.
 *   chunk_offsets uint64[n_chunks + 1]: chunk_offsets[c] = the number of
 *                codewords whose FIRST bit lies before chunk c (subsequences
 *                [c*C, (c+1)*C)), i.e. the output index of the chunk's first
 *                symbol; chunk_offsets[0] = 0, chunk_offsets[n_chunks] =
 *                n_symbols.  These are the output indices of Sec. III-B,
 *                step 3 at chunk granularity, stored by the encoder so that a
 *                gap-array decode needs no device-wide scan (the paper's
 *                decoder derives them by a redundant decoding pass and a
 *                prefix sum, Sec. IV-C).
 *   S = subseq_bits (a multiple of 32), C = chunk_subseqs,
 *   n_subseq = ceil(n_bits / S), n_chunks = ceil(n_subseq / C).
 *
 * Codebooks are canonical (codes of one length are consecutive integers in
 * symbol order, each length's first code continuing the previous length's);
 * lengths[s] = 0 marks a symbol without a codeword.  Codes are right-aligned
 * in uint32.  1 <= max_len <= 32.
 *
 * Symbol widths.  The decoders the paper starts from took one-byte symbols;
 * it adapts them to multi-byte quantization codes (Sec. IV) and notes that
 * the technique carries over to double-precision data (Sec. V-A-3), whose
 * codes can need a wider integer.  A stream's symbols are unsigned integers
 * of symbol_bytes = 1, 2 or 4 bytes (0 is read as 2), and the alphabet must
 * fit the width: alphabet_size <= 256, 65536 or HD_MAX_ALPHABET (2^24).  The
 * bitstream itself does not depend on the width; the width fixes the output
 * array's element type (and so the decoded bytes).  The batched, served,
 * Algorithm-2 and reconstruction entry points take 2-byte symbols only.
 *
 * Conventions for every entry point:
 *   - ownership: the caller owns every buffer; the only library-owned object
 *     is hd_table (created by hd_table_create, freed by hd_table_destroy);
 *   - errors: no exception or abort crosses this interface.  Argument and
 *     format errors are returned synchronously.  Data-dependent faults found
 *     while decoding on the device are reported asynchronously through the
 *     workspace status word (hd_decode_status);
 *   - device calls are asynchronous and ordered on the given hipStream_t
 *     (passed as void*; NULL = the null stream).  Calls on distinct
 *     workspaces may run concurrently; calls sharing a workspace must be
 *     ordered by the caller.
 */
#ifndef HD_H
#define HD_H

#include <stddef.h>
#include <stdint.h>

#define HD_MAX_ALPHABET (1u << 24)

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HD_OK = 0,
    HD_ERR_ARG = -1,          /* bad pointer, size or parameter                  */
    HD_ERR_INFEASIBLE = -2,   /* more used symbols than 2^max_len                */
    HD_ERR_SYMBOL = -3,       /* symbol >= alphabet_size or without a codeword   */
    HD_ERR_CORRUPT = -4,      /* stream/metadata inconsistent with the codebook  */
    HD_ERR_NOMEM = -5,        /* host or device allocation failed                */
    HD_ERR_DEVICE = -6,       /* HIP runtime error                               */
    HD_ERR_UNSUPPORTED = -7   /* valid input this decoder does not take          */
} hd_status;

typedef enum {
    HD_MODE_GAP = 0,          /* start each subsequence from the gap array       */
    HD_MODE_SELF_SYNC = 1     /* find the starts by self-synchronization; reads
                                 neither gap nor chunk_offsets (may be NULL)     */
} hd_mode;

typedef struct {
    uint32_t subseq_bits;     /* S: bits per subsequence, multiple of 32, >= 32  */
    uint32_t chunk_subseqs;   /* C: subsequences per chunk, >= 1                 */
    uint32_t symbol_bytes;    /* width of a symbol: 1, 2 or 4 (0 = 2)            */
} hd_layout;

typedef struct {
    uint64_t n_symbols;       /* n: decoded symbols                              */
    uint64_t n_bits;          /* B: total codeword bits                          */
    uint64_t n_words;         /* units in `words`, guard included                */
    uint64_t n_subseq;        /* K = ceil(B / S)                                 */
    uint64_t n_chunks;        /* M = ceil(K / C)                                 */
    uint32_t subseq_bits;     /* S */
    uint32_t chunk_subseqs;   /* C */
    uint32_t alphabet_size;   /* A */
    uint32_t max_len;         /* L */
    uint32_t symbol_bytes;    /* width of a decoded symbol: 1, 2 or 4 (0 = 2)    */
    uint32_t reserved;        /* set to 0                                        */
} hd_stream_info;

typedef struct hd_table hd_table;

/* Decode-time knobs.  Zero in any field means "choose automatically". */
typedef struct {
    uint32_t waves_per_group; /* wavefronts per workgroup, 1..16 (automatic: the
                                 most wavefronts per CU the LDS footprint allows) */
    uint32_t stage_symbols;   /* LDS output staging per wavefront, in symbols,
                                 a multiple of 64 in [256, 16384]                 */
    uint32_t groups_per_cu;   /* persistent workgroups per compute unit           */
    uint32_t reserved;        /* unused; set to 0                                 */
} hd_tune;

/* A device-resident stream.  All pointers are device memory owned by the
 * caller; `table` must have been created for the stream's codebook. */
typedef struct {
    const uint32_t *words;
    const uint8_t *gap;            /* HD_MODE_GAP only */
    const uint64_t *chunk_offsets; /* HD_MODE_GAP only */
    hd_stream_info info;
    const hd_table *table;
} hd_dstream;

/* ---------------------------------------------------------------- host --- */

/*
 * Optimal length-limited code lengths and canonical codes from a histogram
 * (Sec. II-B: a prefix-free code giving frequent symbols short codewords; the
 * paper leaves the construction to its encoder, this library minimizes the
 * total coded length subject to lengths <= L).
 *   hist[A]    counts per symbol (0 = unused)                       [in]
 *   lengths[A] code length per symbol, 0 for unused                 [out]
 *   codes[A]   right-aligned canonical code per symbol, 0 if unused [out]
 * Ties among optimal length vectors are broken deterministically: symbols are
 * ranked by (count, symbol) and, at equal weight, a single symbol ranks
 * before a merged pair.  One used symbol gets length 1; none gives an empty
 * code.  Returns HD_ERR_INFEASIBLE when more than 2^L symbols are used,
 * HD_ERR_ARG for A outside [1, HD_MAX_ALPHABET] or L outside [1, 32].
 * Synchronous.
 */
hd_status hd_build_codebook(const uint64_t *hist, uint32_t A, uint32_t L,
                            uint8_t *lengths, uint32_t *codes);

/*
 * Reference encoder (host): packs syms[n] (unsigned integers of
 * lay->symbol_bytes bytes each) with the codebook into the stream format
 * above and emits the gap array (Sec. III-C) and the chunk offsets.
 * Two-call use: with words == NULL only *info is filled (sizes, and the
 * symbol width); then call again with buffers of at least info->n_words /
 * n_subseq / n_chunks + 1 entries.  Returns HD_ERR_SYMBOL for a symbol >= A
 * or without a codeword, HD_ERR_ARG for a bad layout (S not a positive
 * multiple of 32, C == 0, a width other than 0, 1, 2, 4), an alphabet that
 * does not fit the width, or short buffers.  The codebook need not be
 * canonical.  Synchronous.
 */
hd_status hd_encode_ref(const void *syms, uint64_t n, const uint8_t *lengths,
                        const uint32_t *codes, uint32_t A, uint32_t L, const hd_layout *lay,
                        uint32_t *words, uint64_t words_cap, uint8_t *gap, uint64_t gap_cap,
                        uint64_t *chunk_offsets, uint64_t chunk_cap, hd_stream_info *info);

/*
 * The stream-format sizes of n_symbols symbols coded in n_bits bits under
 * *lay, alphabet A and length limit L: fills *info (n_words = n_subseq * S /
 * 32 + 2, n_subseq = ceil(n_bits / S), n_chunks = ceil(n_subseq / C); the
 * chunk-offset array has n_chunks + 1 entries; symbol_bytes = the layout's
 * width).  HD_ERR_ARG for a bad layout (S not a positive multiple of 32,
 * C == 0, a width other than 0, 1, 2, 4), an alphabet A that does not fit the
 * width or L outside [1, 32]; HD_ERR_CORRUPT when n_bits is outside
 * [n_symbols, n_symbols * L].
 * Synchronous, host only.
 */
hd_status hd_stream_layout(uint64_t n_symbols, uint64_t n_bits, uint32_t A, uint32_t L, const hd_layout *lay,
                           hd_stream_info *info);

/* --------------------------------------------------------------- device -- */

/*
 * Builds the device-resident decode table of a canonical codebook: a
 * first-level lookup table indexed by the next `lut_bits` stream bits (0 =
 * default, else 6..14, capped at L) giving (symbol, length) for codewords up
 * to that length, plus per-length canonical limits and the symbol list for
 * longer codewords.  The paper keeps its codebook in global memory and relies
 * on the cache (Sec. IV-B); here each workgroup copies the first level and
 * the limits into LDS.  The upload is enqueued on hip_stream; the table may
 * be used by later work on that stream at once.  Alphabets up to
 * HD_MAX_ALPHABET.  Returns HD_ERR_UNSUPPORTED for a non-canonical codebook.
 * *out is owned by the caller until hd_table_destroy.
 */
hd_status hd_table_create(const uint8_t *lengths, const uint32_t *codes, uint32_t A, uint32_t L,
                          uint32_t lut_bits, void *hip_stream, hd_table **out);

/* Frees a table (synchronizes the device first).  NULL is ignored. */
void hd_table_destroy(hd_table *t);

/* Bytes of LDS one workgroup spends on the table (first level + limits). */
size_t hd_table_lds_bytes(const hd_table *t);

/*
 * Device workspace bytes hd_decode needs for stream s in mode m (tune may be
 * NULL).  The workspace holds the status area: a 256-byte header (word 0:
 * status bits of the synchronization phase; word 1: the number of per-
 * wavefront status slots the last decode kernel wrote) and the slots
 * themselves.  In HD_MODE_SELF_SYNC it also holds the output-index scan of
 * the per-tile totals, the found sync points, per-tile records (entry
 * probe results) and the list of tiles left unconverged with its count.  It
 * needs no initialization: every word a call reads is written by that call's
 * kernels first.
 */
hd_status hd_decode_workspace_size(const hd_dstream *s, hd_mode m, const hd_tune *tune,
                                   size_t *bytes);

/*
 * Decodes one stream into out[0 .. n_symbols) (device memory, 16-byte
 * aligned), an array of unsigned integers of info.symbol_bytes bytes (the
 * alphabet must fit that width; HD_ERR_ARG otherwise).
 * HD_MODE_GAP: each subsequence starts at k*S + gap[k] (Sec. III-C); output
 * indices are the stored chunk offsets, refined per subsequence by a
 * wavefront scan of decoded counts (Sec. III-B, step 3); symbols are staged
 * in LDS and written with coalesced stores (Sec. IV-B, Algorithm 1).  One
 * kernel launch.
 * HD_MODE_SELF_SYNC: the sync point of every subsequence is found by
 * decoding from the raw boundary until the path meets the previous
 * subsequence's verified exit (Sec. III-B-2, steps 1-2), the counts found on
 * the way are scanned (step 3) and the decode/write step is the same as in
 * gap mode (step 4).  No gap or chunk_offsets input is read.
 * Asynchronous on hip_stream.  Returns HD_ERR_ARG / HD_ERR_UNSUPPORTED for
 * bad arguments (including a workspace smaller than
 * hd_decode_workspace_size), HD_ERR_DEVICE for launch failures.  Faults in
 * the data are reported by hd_decode_status.
 */
hd_status hd_decode(const hd_dstream *s, void *out, hd_mode m, const hd_tune *tune,
                    void *workspace, size_t ws_bytes, void *hip_stream);

/*
 * hd_decode in two parts, for callers that time the phases or decode one
 * stream repeatedly.  hd_decode_prepare enqueues the output-index phase
 * (gap mode: nothing, the offsets are stored in the stream; self-sync mode:
 * the synchronization steps 1-3 of Sec. III-B-2) and leaves its result in the
 * workspace; hd_decode_run enqueues the decode-and-write step (step 4,
 * Sec. IV-B) reading that result.  prepare followed by run on one stream
 * equals hd_decode; run may be repeated while the workspace is untouched.
 * Same arguments, errors and asynchrony as hd_decode.
 */
hd_status hd_decode_prepare(const hd_dstream *s, hd_mode m, const hd_tune *tune, void *workspace,
                            size_t ws_bytes, void *hip_stream);
hd_status hd_decode_run(const hd_dstream *s, void *out, hd_mode m, const hd_tune *tune,
                        void *workspace, size_t ws_bytes, void *hip_stream);

/*
 * After hd_decode_prepare (or hd_decode) in HD_MODE_SELF_SYNC on this
 * workspace: copies the synchronization point found for every subsequence,
 * relative to the subsequence start (the gap-array convention), into
 * gap_out[0 .. n_subseq) (device memory), asynchronously on hip_stream.  The
 * gap array holds exactly what self-synchronization finds (Sec. III-C), so a
 * plain Huffman stream can be synchronized once and decoded in HD_MODE_GAP
 * afterwards.  HD_ERR_ARG for a workspace smaller than the self-sync size.
 */
hd_status hd_decode_sync_points(const hd_dstream *s, const void *workspace, size_t ws_bytes,
                                uint8_t *gap_out, void *hip_stream);

/*
 * Workspace bytes for hd_decode_batch over n_streams streams (gap mode).
 */
hd_status hd_decode_batch_workspace_size(const hd_dstream *streams, uint32_t n_streams,
                                         hd_mode m, size_t *bytes);

/*
 * Decodes n_streams independent streams, each with its own table, layout and
 * alphabet, into outs[i] (device memory, n_symbols of stream i, 16-byte
 * aligned) with one persistent decode launch.  The paper groups sequences by compression ratio and launches one
 * kernel per group, each with its own shared-memory size (Sec. IV-C, Alg. 2);
 * here workgroups walk (stream, group of tiles) items of every stream and
 * reload the LDS decode table only when the stream changes.  The launch's LDS
 * layout reserves the largest table, subsequence and staging of the batch.
 * per_stream, when not NULL, holds n_streams tunes: stage_symbols of each
 * stream, and the launch's waves_per_group and groups_per_cu from
 * per_stream[0] (0: the most resident wavefronts the layout allows).  A zero
 * (or absent) stage_symbols takes the stream's need from its mean code length,
 * capped for the batch at the larger of the staging that keeps 16 wavefronts
 * resident per CU and the symbol-weighted median need; tiles above the cap
 * are written in passes.  m must be HD_MODE_GAP (HD_ERR_UNSUPPORTED otherwise);
 * HD_ERR_UNSUPPORTED also when the layout exceeds a workgroup's LDS.
 * Per-call descriptors are uploaded through library-owned pinned staging,
 * without a host wait.  Asynchronous on hip_stream; the status word
 * (hd_decode_status) covers every stream of the batch.
 */
hd_status hd_decode_batch(const hd_dstream *streams, uint32_t n_streams, uint16_t *const *outs,
                          hd_mode m, const hd_tune *per_stream, void *workspace, size_t ws_bytes,
                          void *hip_stream);

/*
 * The paper's shared-memory optimization, literally (Sec. IV-C, Algorithm 2),
 * kept as an ablation beside hd_decode's single persistent launch.  Gap mode
 * only.  Each wavefront tile (64 subsequences) is a "sequence": its
 * compression ratio (16 bits per symbol over its input bits; the symbol count
 * comes from the stored chunk offsets) is classified into T_high + 1 groups,
 * (0,1], ..., (T_high - 1, T_high] and above T_high; on the device the
 * classes are histogrammed and the tile indices key-value sorted by class;
 * the histogram is copied to the host (the call waits for hip_stream here),
 * which prefix-sums it and launches one decode kernel per non-empty class on
 * its own library-owned stream (default priority), each with the staging of
 * its class's upper bound (4 S c + 64 symbols per tile; the last class takes
 * T_high's and writes larger tiles in passes).  T_high is the largest class
 * whose layout still keeps a quarter of a CU's wavefront slots resident (the
 * paper's 25 % occupancy rule).  hip_stream waits for every class launch, so
 * later work on it is ordered after the decode.  The status word
 * (hd_decode_status) covers all launches.  *report (may be NULL) receives
 * T_high, the host time from entry until the histogram is on the host
 * (classification overhead, including the wait for earlier work on
 * hip_stream) and, per class, the tiles, staging and waves per workgroup.
 * Same argument errors as hd_decode.
 */
typedef struct {
    uint32_t t_high;
    uint32_t launches;
    double classify_us;
    uint32_t tiles[17];
    uint32_t stage_symbols[17];
    uint32_t waves_per_group[17];
} hd_cr_classes;

hd_status hd_decode_cr_classes_workspace_size(const hd_dstream *s, size_t *bytes);
hd_status hd_decode_cr_classes(const hd_dstream *s, uint16_t *out, void *workspace, size_t ws_bytes,
                               void *hip_stream, hd_cr_classes *report);

/*
 * Decode-parameter autotuning on a sample stream.  The paper tunes the
 * shared-memory buffer per call from each sequence's compression ratio
 * (Sec. IV-C, Alg. 2, Table I) and compares against a brute-force sweep;
 * here the sweep itself is the tuner, run once per stream class and cached
 * by the caller: hd_decode_run is timed with HIP events (median of three
 * after a warm-up) for waves_per_group in {the occupancy choice, 4, 8, 16}
 * times staging sizes of 0.5x .. 2x the expected tile output, and the fastest
 * tune goes to *best (its time to *best_ms when not NULL).  out and workspace are as for
 * hd_decode on this sample (their contents are overwritten).  Synchronous:
 * waits for hip_stream.
 */
hd_status hd_autotune(const hd_dstream *sample, hd_mode m, void *out, void *workspace,
                      size_t ws_bytes, void *hip_stream, hd_tune *best, float *best_ms);

/*
 * Waits for hip_stream, then reads the status the last decode on this
 * workspace left (the header word and every slot the decode kernel wrote):
 * HD_OK, or HD_ERR_CORRUPT when a lane met an invalid codeword, a
 * subsequence ended off its successor's start, a chunk's decoded count
 * differed from its chunk offsets, the offsets did not start at 0 and end at
 * n_symbols, or self-synchronization found no consistent sync point.
 */
hd_status hd_decode_status(const void *workspace, void *hip_stream);

/*
 * The raw status bits behind hd_decode_status (0 = clean; 0xffffffff when the
 * word could not be read).  Bit 0: a gap byte beyond any codeword length;
 * 1: a window matching no codeword; 2: a subsequence ending off its
 * successor's start; 3: a chunk's decoded count differing from its offsets;
 * 4: chunk offsets not starting at 0 or not ending at n_symbols (self-sync:
 * found counts not adding up to n_symbols); 5: an output index outside
 * [0, n_symbols); 6: self-synchronization found no consistent sync point
 * (the synchronized path from bit 0 does not end on bit n_bits); 7: a code-0
 * position missing from the outlier list (hd_lorenzo_reconstruct).  Waits
 * for hip_stream first.
 */
uint32_t hd_decode_status_bits(const void *workspace, void *hip_stream);

/*
 * hd_decode without a caller workspace and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The workspace is a
 * fixed library array of HD_NOALLOC_SCRATCH_BYTES in device memory (one per
 * GPU, held until the process ends, set up on the first call on each device);
 * streams whose hd_decode_workspace_size exceeds it are refused with
 * HD_ERR_UNSUPPORTED before anything is enqueued.  The call enqueues
 * hd_decode's kernels on hip_stream, then writes the raw status bits (the
 * value hd_decode_status_bits would return for a workspace) into *status, a
 * caller-owned uint32 in device memory, with a plain store: no clearing
 * needed, no host wait.  The array keeps the last call's contents; every
 * word a call reads is written by that call first.  Calls that overlap on one
 * GPU (different streams or threads without ordering) share the array and
 * race: order them.  Same argument errors as hd_decode, plus HD_ERR_ARG for a
 * NULL status.
 */
#define HD_NOALLOC_SCRATCH_BYTES (32u << 20)
hd_status hd_decode_noalloc(const hd_dstream *s, void *out, hd_mode m, const hd_tune *tune,
                            uint32_t *status, void *hip_stream);

/* ------------------------------------------------------------ encoding -- */

/*
 * Device-side encoding into the stream format above: the same words, gap
 * array (Sec. III-C) and chunk offsets as hd_encode_ref, bit for bit.  All
 * buffers are device memory owned by the caller; calls are asynchronous on
 * hip_stream except hd_encode_bits.
 *
 * hd_histogram: hist[A] (uint64, device) = count of each symbol value < A in
 *   syms[n]; the call zeroes hist first.  Values >= A are not counted.
 *   HD_ERR_ARG for A outside [1, 65536] or NULL buffers.
 * hd_encode_workspace_size: bytes of workspace for n symbols with codes of at
 *   most L bits under *lay (0 for a bad layout or L outside [1, 32]).
 * hd_encode_plan: the total codeword bits of syms[n] under lengths[A] (device
 *   uint8), kept in the workspace; flags a symbol >= A or of length 0.
 * hd_encode_bits: waits for hip_stream and returns the planned total in
 *   *n_bits; HD_ERR_SYMBOL when a symbol had no codeword.  The caller sizes
 *   the outputs from it: n_subseq = ceil(n_bits / S), n_chunks =
 *   ceil(n_subseq / C), n_words = n_subseq * S / 32 + 2.
 * hd_encode_write: packs syms[n] with lengths[A] / codes[A] (device, codes
 *   right-aligned) into words[n_words] (zero-filled by the call, guard units
 *   included), gap[n_subseq] and chunk_offsets[n_chunks + 1].  Needs the plan of
 *   the same symbols in the same workspace.  HD_ERR_ARG for a bad layout,
 *   n_chunks != ceil(n_subseq / C), a workspace below
 *   hd_encode_workspace_size or NULL buffers.  A unit index beyond n_words
 *   sets status bit 5 (hd_decode_status_bits reads the workspace's status
 *   word) instead of writing.
 */
hd_status hd_histogram(const uint16_t *syms, uint64_t n, uint32_t A, uint64_t *hist, void *hip_stream);

/*
 * The codebook of hd_build_codebook, built on the device from a device
 * histogram: lengths[A] (uint8) and codes[A] (uint32, right-aligned), device
 * memory, byte for byte what hd_build_codebook returns for the same counts
 * (optimal lengths <= L by package-merge, ties ranked by (count, symbol) with
 * a symbol ahead of a pair of equal weight; canonical codes).  The paper
 * takes the codebook from its encoder's GPU builder (Sec. II-B, Sec. VI); this
 * keeps a device encode (hd_histogram, this call, hd_encode_plan/_write) free
 * of host round trips.  One workgroup builds it in LDS: at most 4096 used
 * symbols, A <= 65536 (HD_ERR_UNSUPPORTED above), counts below 2^40.  Data-
 * dependent failures are reported through the workspace status word
 * (hd_decode_status_bits(workspace)): bit 8 more used symbols than 2^L,
 * bit 9 more than 4096 used symbols, bit 10 a count of 2^40 or more; the
 * codebook is then all zero.  workspace: hd_codebook_workspace_size(L) bytes,
 * 256-byte aligned, no initialization.  Asynchronous on hip_stream.
 */
size_t hd_codebook_workspace_size(uint32_t L);
hd_status hd_build_codebook_device(const uint64_t *hist, uint32_t A, uint32_t L, uint8_t *lengths,
                                   uint32_t *codes, void *workspace, size_t ws_bytes, void *hip_stream);

size_t hd_encode_workspace_size(uint64_t n, uint32_t L, const hd_layout *lay);
hd_status hd_encode_plan(const uint16_t *syms, uint64_t n, const uint8_t *lengths, uint32_t A, void *workspace,
                         size_t ws_bytes, void *hip_stream);
hd_status hd_encode_bits(const void *workspace, uint64_t *n_bits, void *hip_stream);
hd_status hd_encode_write(const uint16_t *syms, uint64_t n, const uint8_t *lengths, const uint32_t *codes,
                          uint32_t A, const hd_layout *lay, uint32_t *words, uint64_t n_words, uint8_t *gap,
                          uint64_t n_subseq, uint64_t *chunk_offsets, uint64_t n_chunks, void *workspace,
                          size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------ reconstruction -- */

/*
 * SZ-style reconstruction of the field behind decoded quantization codes (the
 * step after Huffman decoding in the cuSZ decompression of Sec. V-B-2; the
 * error-bounded scheme of Sec. II-A).  The codes are the first-order 3-D
 * Lorenzo prediction residuals of the prequantized integer field q, shifted
 * by radius, with code 0 marking a residual held in the outlier list:
 *
 *   r = code - radius, or outlier_val[m] where code == 0 and
 *       outlier_idx[m] is the position's flat index;
 *   q(i,j,k) = sum of r over [0,i] x [0,j] x [0,k] (inverse Lorenzo);
 *   out(i,j,k) = (float)((double)q * (2.0 * eb)).
 *
 * codes      device uint16[ni*nj*nk], C order (k fastest): ni planes of nj
 *            rows of nk values.  2-D fields pass ni = 1, 1-D fields ni = nj = 1.
 * outlier_idx, outlier_val
 *            device uint64[n_outliers] strictly ascending flat indices and
 *            int32 residuals.  Only code-0 positions consult the list; an entry
 *            at a non-zero code is ignored.  An unsorted list gives unspecified
 *            values (no access outside the list).  NULL when n_outliers = 0.
 * out        device float32[ni*nj*nk]; also the kernels' int32 scratch.
 * q_out      optional device int32[ni*nj*nk] for q itself (NULL to skip).
 * workspace  device memory of hd_lorenzo_workspace_size(ni, nj, nk) bytes,
 *            16-byte aligned; its first word is a status word that
 *            hd_decode_status / hd_decode_status_bits read like a decode's
 *            (bit 7: a code-0 position missing from the outlier list; its
 *            value then counts as 0).  The call clears it on the device.
 *
 * Every q must fit int32 (partial sums wrap modulo 2^32 and still end exact).
 * Returns HD_ERR_ARG for NULL buffers, a short or misaligned workspace,
 * radius 0 or eb not positive and finite; HD_ERR_UNSUPPORTED for nk > 4096
 * unless ni = nj = 1 (a 1-D field of any length up to 2^32 - 1).
 * An empty field (a zero extent) only clears the status word.  Asynchronous
 * on hip_stream; HD_ERR_DEVICE for launch failures.
 */
size_t hd_lorenzo_workspace_size(uint32_t ni, uint32_t nj, uint32_t nk);
hd_status hd_lorenzo_reconstruct(const uint16_t *codes, uint32_t ni, uint32_t nj, uint32_t nk,
                                 uint32_t radius, const uint64_t *outlier_idx, const int32_t *outlier_val,
                                 uint64_t n_outliers, double eb, float *out, int32_t *q_out, void *workspace,
                                 size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------- serving -- */

/*
 * A decode server with continuous batching (no counterpart in the paper,
 * which measures single calls).  It owns one device arena of hbm_budget
 * bytes; every admitted request's output (n_symbols uint16) and every
 * batch's workspace come from it, so the in-flight device footprint never
 * exceeds the budget.  A scheduler thread admits queued requests in arrival
 * order while they fit, launches each admitted group as one hd_decode_batch
 * on one of n_hip_streams streams (default priority), and retires batches by
 * event.  Requests arriving while batches run are admitted as memory and
 * stream slots free up; their work overlaps on the device.  Request streams
 * (device buffers and tables) must stay alive until the request completes.
 */
typedef struct hd_server hd_server;

hd_status hd_server_create(size_t hbm_budget, uint32_t n_hip_streams, uint32_t max_batch,
                           hd_server **out);
/* Waits for running batches, drops requests never admitted, frees the arena. */
void hd_server_destroy(hd_server *s);
/* Queues a gap-mode decode of *stream; HD_ERR_NOMEM when its output plus
 * workspace exceed the whole budget (it could never be admitted). */
hd_status hd_server_submit(hd_server *s, const hd_dstream *stream, uint64_t *request_id);
/* Non-blocking: up to cap ids of requests completed since the last poll. */
hd_status hd_server_poll(hd_server *s, uint64_t *done_ids, uint32_t cap, uint32_t *n_done);
/* A completed request: device output (valid until release), its batch's
 * decode status, and submit/completion times in seconds (steady clock). */
hd_status hd_server_result(hd_server *s, uint64_t id, const uint16_t **out, hd_status *status,
                           double *t_submit, double *t_done);
/* Returns a completed request's output memory to the arena. */
hd_status hd_server_release(hd_server *s, uint64_t id);
hd_status hd_server_stats(hd_server *s, uint64_t *n_batches, uint64_t *n_done, uint64_t *queued,
                          uint64_t *arena_used, uint64_t *arena_peak);

/* Static description of a status code. */
const char *hd_status_str(hd_status s);

#ifdef __cplusplus
}
#endif

#endif /* HD_H */
