/*
 * hdref.c -- CPU ORACLE FOR CANONICAL-HUFFMAN CODING OF QUANTIZATION CODES
 * (uint16 symbols; the _w entry points also take uint8 and uint32 symbols).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  The product
 * library shares no code, header, table or helper with it.
 *
 * Every routine here is the plain definition of what it computes, written for
 * a reader to check by eye, not for speed:
 *
 *   hdref_histogram        symbol counts (Sec. II-B: frequent symbols get
 *                          short codewords, so the counts drive the code).
 *   hdref_code_lengths     optimal length-limited code lengths by
 *                          package-merge (Larmore & Hirschberg, 1990).  The
 *                          paper does not say how its codebook is built; it
 *                          only requires a prefix-free Huffman code (Sec. II-B).
 *   hdref_canonical_codes  canonical codeword assignment (codes of one length
 *                          are consecutive integers in symbol order; the first
 *                          code of each length continues the previous one).
 *   hdref_encode           MSB-first packing into 32-bit units (Sec. III-B:
 *                          units are unsigned 32-bit numbers holding the
 *                          codewords), plus the gap array (Sec. III-C: one
 *                          byte per subsequence telling a thread where the
 *                          first decodable codeword begins) and the per-chunk
 *                          symbol counts a decoder needs for output indices
 *                          (Sec. III-B, step 3).
 *   hdref_decode           bit-serial prefix-tree decoding, one bit at a time
 *                          (the behaviour of the baseline decoder, Sec. III-A),
 *                          for ANY prefix code, canonical or not.
 *   hdref_decode_from      the same decoder started at a known codeword start
 *                          (a gap-array entry), for chunk-parallel timing.
 *   hdref_selfsync         true synchronization points and per-subsequence
 *                          counts (Sec. III-B: one sync point per subsequence;
 *                          the count of valid codewords per subsequence feeds
 *                          the prefix sum), and a simulation of how far a
 *                          decoder started on a raw subsequence boundary runs
 *                          before it lands on a true codeword boundary
 *                          (Sec. III-B-1, self-synchronization).
 *   hdref_gap_backward     the gap array in the signed, backward form of the
 *                          paper's Fig. 1 example (offset to the start of the
 *                          codeword that straddles the boundary).
 *
 * Conventions (readings of points the paper leaves open):
 *   - stream bit i is bit (31 - i % 32) of unit i / 32 (MSB first);
 *   - a codeword belongs to the subsequence holding its FIRST bit;
 *   - gap[k] = p_k - k*S where p_k is the first codeword start >= k*S, the end
 *     of the stream counting as a start (forward, in bits);
 *   - the unit array holds ceil(K*S/32) + 2 units, K = ceil(B/S); the tail
 *     is zero (the product format takes S as a multiple of 32; the oracle
 *     accepts any S >= 1 so that the paper's 8-bit Fig. 1 example applies).
 *
 * Return codes: 0 ok, -1 bad argument, -2 infeasible (more used symbols than
 * 2^L), -3 symbol out of range or without a codeword, -4 corrupt stream or
 * inconsistent code, -5 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HDREF_OK 0
#define HDREF_EARG (-1)
#define HDREF_EINFEASIBLE (-2)
#define HDREF_ESYMBOL (-3)
#define HDREF_ECORRUPT (-4)
#define HDREF_ENOMEM (-5)

/* ------------------------------------------------------------------------ */
/* Symbol widths                                                             */
/* ------------------------------------------------------------------------ */
/*
 * The original decoders took one-byte symbols; the paper adapts them to
 * multi-byte quantization codes (Sec. IV) and notes that the same holds for
 * double-precision data (Sec. V-A-3), whose codes can need a wider integer.
 * A symbol array here holds unsigned integers of 1, 2 or 4 bytes; the
 * alphabet must fit the width: at most 2^8, 2^16 or HDREF_MAX_ALPHABET
 * symbols.  The 16-bit entry points are the width-2 case.
 */
#define HDREF_MAX_ALPHABET (1u << 24)

static int width_fits(uint32_t width, uint32_t A)
{
    if (A == 0)
        return 0;
    if (width == 1)
        return A <= 256u;
    if (width == 2)
        return A <= 65536u;
    if (width == 4)
        return A <= HDREF_MAX_ALPHABET;
    return 0;
}

static uint32_t sym_get(const void *x, uint32_t width, uint64_t i)
{
    if (width == 1)
        return ((const uint8_t *)x)[i];
    if (width == 2)
        return ((const uint16_t *)x)[i];
    return ((const uint32_t *)x)[i];
}

static void sym_set(void *out, uint32_t width, uint64_t i, uint32_t v)
{
    if (width == 1)
        ((uint8_t *)out)[i] = (uint8_t)v;
    else if (width == 2)
        ((uint16_t *)out)[i] = (uint16_t)v;
    else
        ((uint32_t *)out)[i] = v;
}

/* ------------------------------------------------------------------------ */
/* Histogram                                                                 */
/* ------------------------------------------------------------------------ */

int hdref_histogram_w(const void *x, uint32_t width, uint64_t n, uint32_t A, uint64_t *cnt)
{
    if (!width_fits(width, A) || (n > 0 && x == NULL) || cnt == NULL)
        return HDREF_EARG;
    for (uint32_t s = 0; s < A; ++s)
        cnt[s] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t v = sym_get(x, width, i);
        if (v >= A)
            return HDREF_ESYMBOL;
        cnt[v] += 1;
    }
    return HDREF_OK;
}

int hdref_histogram(const uint16_t *x, uint64_t n, uint32_t A, uint64_t *cnt)
{
    return hdref_histogram_w(x, 2, n, A, cnt);
}

/* ------------------------------------------------------------------------ */
/* Package-merge                                                             */
/* ------------------------------------------------------------------------ */
/*
 * Coin-collector formulation.  Every used symbol owns one coin of each
 * denomination 2^-1 .. 2^-L whose numismatic value is the symbol's count.
 * The cheapest set of coins with total denomination (m - 1) gives the optimal
 * code subject to lengths <= L; a symbol's code length is the number of its
 * coins in that set.  Procedure:
 *   list(L)   = the leaves, sorted by (count, symbol);
 *   list(d)   = merge(leaves, packages of consecutive pairs of list(d+1)),
 *               d = L-1 .. 1, a leaf placed before a package of equal value;
 *   selection = the first 2m - 2 items of list(1);
 *   len(s)    = number of leaves of s reached by expanding the selection.
 */

typedef struct {
    uint64_t w;
    int32_t sym;        /* >= 0: a leaf (coin) of this symbol; -1: package */
    int32_t a, b;       /* package: indices of its two items in the pool   */
} pm_node;

typedef struct {
    uint64_t w;
    uint32_t sym;
} pm_leaf;

static int pm_leaf_cmp(const void *pa, const void *pb)
{
    const pm_leaf *x = (const pm_leaf *)pa, *y = (const pm_leaf *)pb;
    if (x->w != y->w)
        return x->w < y->w ? -1 : 1;
    return x->sym < y->sym ? -1 : (x->sym > y->sym ? 1 : 0);
}

int hdref_code_lengths(const uint64_t *cnt, uint32_t A, uint32_t L, uint8_t *len)
{
    if (cnt == NULL || len == NULL || A == 0 || A > HDREF_MAX_ALPHABET || L < 1 || L > 32)
        return HDREF_EARG;
    uint32_t m = 0;
    for (uint32_t s = 0; s < A; ++s) {
        len[s] = 0;
        if (cnt[s] > 0)
            ++m;
    }
    if (m == 0)
        return HDREF_OK;
    if (m == 1) {                     /* a lone symbol still needs one bit */
        for (uint32_t s = 0; s < A; ++s)
            if (cnt[s] > 0)
                len[s] = 1;
        return HDREF_OK;
    }
    if (L < 32 && (uint64_t)m > ((uint64_t)1 << L))
        return HDREF_EINFEASIBLE;

    pm_leaf *leaves = (pm_leaf *)malloc(sizeof(pm_leaf) * m);
    uint64_t pool_cap = (uint64_t)m + (uint64_t)m * L;  /* leaves + packages */
    pm_node *pool = (pm_node *)malloc(sizeof(pm_node) * pool_cap);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * 2 * m);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * 2 * m);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (2 * (uint64_t)m * (L + 1) + 8));
    if (!leaves || !pool || !cur || !nxt || !stack) {
        free(leaves); free(pool); free(cur); free(nxt); free(stack);
        return HDREF_ENOMEM;
    }
    uint32_t j = 0;
    for (uint32_t s = 0; s < A; ++s)
        if (cnt[s] > 0) {
            leaves[j].w = cnt[s];
            leaves[j].sym = s;
            ++j;
        }
    qsort(leaves, m, sizeof(pm_leaf), pm_leaf_cmp);

    /* pool[0..m) are the leaves, shared by all levels. */
    uint64_t np = 0;
    for (uint32_t i = 0; i < m; ++i) {
        pool[np].w = leaves[i].w;
        pool[np].sym = (int32_t)leaves[i].sym;
        pool[np].a = pool[np].b = -1;
        ++np;
    }

    /* list(L) = leaves */
    uint32_t ncur = m;
    for (uint32_t i = 0; i < m; ++i)
        cur[i] = (int32_t)i;

    for (uint32_t d = L - 1; d >= 1; --d) {
        /* packages of consecutive pairs of list(d+1); an odd last item is dropped */
        uint32_t npk = ncur / 2;
        uint64_t pk0 = np;
        for (uint32_t p = 0; p < npk; ++p) {
            pool[np].w = pool[cur[2 * p]].w + pool[cur[2 * p + 1]].w;
            pool[np].sym = -1;
            pool[np].a = cur[2 * p];
            pool[np].b = cur[2 * p + 1];
            ++np;
        }
        /* merge leaves with the packages; equal values: leaf first */
        uint32_t li = 0, pi = 0, o = 0;
        while (li < m || pi < npk) {
            int take_leaf;
            if (li >= m)
                take_leaf = 0;
            else if (pi >= npk)
                take_leaf = 1;
            else
                take_leaf = pool[li].w <= pool[pk0 + pi].w;
            nxt[o++] = take_leaf ? (int32_t)li++ : (int32_t)(pk0 + pi++);
        }
        int32_t *t = cur; cur = nxt; nxt = t;
        ncur = o;
        if (d == 1)
            break;
    }
    if (L == 1) {
        /* list(1) is just the leaves: only m == 2 is feasible (checked above) */
    }

    /* expand the first 2m-2 items of list(1) and count the leaves reached */
    uint32_t nsel = 2 * m - 2;
    if (nsel > ncur) {                 /* cannot happen when m <= 2^L */
        free(leaves); free(pool); free(cur); free(nxt); free(stack);
        return HDREF_EINFEASIBLE;
    }
    uint32_t *depth = (uint32_t *)calloc(A, sizeof(uint32_t));
    if (!depth) {
        free(leaves); free(pool); free(cur); free(nxt); free(stack);
        return HDREF_ENOMEM;
    }
    for (uint32_t i = 0; i < nsel; ++i) {
        int64_t sp = 0;
        stack[sp++] = cur[i];
        while (sp > 0) {
            int32_t v = stack[--sp];
            if (pool[v].sym >= 0) {
                depth[pool[v].sym] += 1;
            } else {
                stack[sp++] = pool[v].a;
                stack[sp++] = pool[v].b;
            }
        }
    }
    int rc = HDREF_OK;
    for (uint32_t s = 0; s < A; ++s) {
        if (depth[s] > L)
            rc = HDREF_ECORRUPT;
        len[s] = (uint8_t)depth[s];
    }
    free(depth); free(leaves); free(pool); free(cur); free(nxt); free(stack);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Canonical codes                                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint8_t len;
    uint32_t sym;
} cc_item;

static int cc_cmp(const void *pa, const void *pb)
{
    const cc_item *x = (const cc_item *)pa, *y = (const cc_item *)pb;
    if (x->len != y->len)
        return x->len < y->len ? -1 : 1;
    return x->sym < y->sym ? -1 : (x->sym > y->sym ? 1 : 0);
}

/* Sort the used symbols by (length, symbol).  The first gets the all-zero
 * code; each next one gets (previous + 1) shifted left by the length step.
 * Codes are right-aligned in uint32.  Unused symbols get code 0. */
int hdref_canonical_codes(const uint8_t *len, uint32_t A, uint32_t *code)
{
    if (len == NULL || code == NULL || A == 0 || A > HDREF_MAX_ALPHABET)
        return HDREF_EARG;
    cc_item *it = (cc_item *)malloc(sizeof(cc_item) * A);
    if (!it)
        return HDREF_ENOMEM;
    uint32_t m = 0;
    for (uint32_t s = 0; s < A; ++s) {
        code[s] = 0;
        if (len[s] > 32) {
            free(it);
            return HDREF_EARG;
        }
        if (len[s] > 0) {
            it[m].len = len[s];
            it[m].sym = s;
            ++m;
        }
    }
    qsort(it, m, sizeof(cc_item), cc_cmp);
    uint64_t c = 0;
    for (uint32_t i = 0; i < m; ++i) {
        if (i > 0)
            c = (c + 1) << (it[i].len - it[i - 1].len);
        if (c >> it[i].len) {          /* more codes than the lengths allow */
            free(it);
            return HDREF_ECORRUPT;
        }
        code[it[i].sym] = (uint32_t)c;
    }
    free(it);
    return HDREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Encoder                                                                   */
/* ------------------------------------------------------------------------ */

static void put_bit(uint32_t *words, uint64_t pos, unsigned bit)
{
    if (bit)
        words[pos >> 5] |= (uint32_t)1 << (31 - (pos & 31));
}

static unsigned get_bit(const uint32_t *words, uint64_t pos)
{
    return (words[pos >> 5] >> (31 - (pos & 31))) & 1u;
}

/*
 * info[0] = B (total code bits), info[1] = number of 32-bit units,
 * info[2] = K (subsequences), info[3] = M (chunks).
 * With words == NULL only info is filled (size query).
 */
int hdref_encode_w(const void *x, uint32_t width, uint64_t n, const uint8_t *len, const uint32_t *code,
                   uint32_t A, uint32_t S, uint32_t C,
                   uint32_t *words, uint64_t words_cap, uint8_t *gap, uint64_t gap_cap,
                   uint32_t *chunk_counts, uint64_t chunk_cap, uint64_t *info)
{
    if ((n > 0 && x == NULL) || len == NULL || code == NULL || info == NULL)
        return HDREF_EARG;
    if (!width_fits(width, A) || S == 0 || C == 0)
        return HDREF_EARG;
    uint64_t B = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t v = sym_get(x, width, i);
        if (v >= A || len[v] == 0)
            return HDREF_ESYMBOL;
        B += len[v];
    }
    uint64_t K = (B + S - 1) / S;
    uint64_t M = (K + C - 1) / C;
    uint64_t NW = (K * S + 31) / 32 + 2;
    info[0] = B;
    info[1] = NW;
    info[2] = K;
    info[3] = M;
    if (words == NULL)
        return HDREF_OK;
    if (words_cap < NW || gap_cap < K || chunk_cap < M || (K > 0 && (gap == NULL || chunk_counts == NULL)))
        return HDREF_EARG;

    memset(words, 0, NW * sizeof(uint32_t));
    for (uint64_t c = 0; c < M; ++c)
        chunk_counts[c] = 0;

    uint64_t pos = 0;      /* start of the next codeword            */
    uint64_t kb = 0;       /* next subsequence boundary to resolve  */
    for (uint64_t i = 0; i < n; ++i) {
        /* every boundary k*S in (previous start, pos] has p_k = pos */
        while (kb < K && kb * S <= pos) {
            gap[kb] = (uint8_t)(pos - kb * S);
            ++kb;
        }
        chunk_counts[(pos / S) / C] += 1;
        uint32_t v = sym_get(x, width, i);
        unsigned l = len[v];
        uint32_t cw = code[v];
        for (unsigned b = 0; b < l; ++b)            /* MSB of the codeword first */
            put_bit(words, pos + b, (cw >> (l - 1 - b)) & 1u);
        pos += l;
    }
    /* the end of the stream counts as a codeword start */
    while (kb < K) {
        gap[kb] = (uint8_t)(B - kb * S);
        ++kb;
    }
    return HDREF_OK;
}

int hdref_encode(const uint16_t *x, uint64_t n, const uint8_t *len, const uint32_t *code,
                 uint32_t A, uint32_t S, uint32_t C,
                 uint32_t *words, uint64_t words_cap, uint8_t *gap, uint64_t gap_cap,
                 uint32_t *chunk_counts, uint64_t chunk_cap, uint64_t *info)
{
    return hdref_encode_w(x, 2, n, len, code, A, S, C, words, words_cap, gap, gap_cap, chunk_counts,
                          chunk_cap, info);
}

/* ------------------------------------------------------------------------ */
/* Prefix tree for arbitrary (length, code) pairs                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t child[2];
    int32_t sym;          /* >= 0 at a leaf */
} tr_node;

typedef struct {
    tr_node *nodes;
    uint64_t n, cap;
} tr_tree;

static int tr_new(tr_tree *t)
{
    if (t->n == t->cap) {
        uint64_t nc = t->cap ? 2 * t->cap : 64;
        tr_node *p = (tr_node *)realloc(t->nodes, nc * sizeof(tr_node));
        if (!p)
            return -1;
        t->nodes = p;
        t->cap = nc;
    }
    t->nodes[t->n].child[0] = t->nodes[t->n].child[1] = -1;
    t->nodes[t->n].sym = -1;
    return (int)(t->n++);
}

/* Builds the tree; returns -1 when the code is not prefix-free. */
static int tr_build(tr_tree *t, const uint8_t *len, const uint32_t *code, uint32_t A)
{
    t->nodes = NULL;
    t->n = t->cap = 0;
    if (tr_new(t) < 0)
        return HDREF_ENOMEM;
    for (uint32_t s = 0; s < A; ++s) {
        unsigned l = len[s];
        if (l == 0)
            continue;
        if (l > 32)
            return HDREF_EARG;
        int32_t v = 0;
        for (unsigned b = 0; b < l; ++b) {
            unsigned bit = (code[s] >> (l - 1 - b)) & 1u;
            if (t->nodes[v].sym >= 0)
                return HDREF_ECORRUPT;           /* a shorter codeword is a prefix */
            if (t->nodes[v].child[bit] < 0) {
                int nv = tr_new(t);
                if (nv < 0)
                    return HDREF_ENOMEM;
                t->nodes[v].child[bit] = nv;
            }
            v = t->nodes[v].child[bit];
        }
        if (t->nodes[v].sym >= 0 || t->nodes[v].child[0] >= 0 || t->nodes[v].child[1] >= 0)
            return HDREF_ECORRUPT;               /* duplicate or prefix of another */
        t->nodes[v].sym = (int32_t)s;
    }
    return HDREF_OK;
}

/* Decodes one codeword starting at *pos.  Returns the symbol, -1 when the
 * walk leaves the tree, -2 when it runs past `limit` bits. */
static int64_t tr_step(const tr_tree *t, const uint32_t *words, uint64_t *pos, uint64_t limit)
{
    int32_t v = 0;
    while (t->nodes[v].sym < 0) {
        if (*pos >= limit)
            return -2;
        unsigned bit = get_bit(words, *pos);
        *pos += 1;
        v = t->nodes[v].child[bit];
        if (v < 0)
            return -1;
    }
    return t->nodes[v].sym;
}

/* ------------------------------------------------------------------------ */
/* Bit-serial decoder                                                        */
/* ------------------------------------------------------------------------ */

/* Decodes exactly n symbols from bit 0 and requires the stream to end at
 * bit B.  words must hold at least ceil(B/32) units. */
int hdref_decode_w(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n,
                   const uint8_t *len, const uint32_t *code, uint32_t A, void *out, uint32_t width)
{
    if (len == NULL || code == NULL || !width_fits(width, A) || (n > 0 && (out == NULL || words == NULL)))
        return HDREF_EARG;
    if (n_words * 32 < B)
        return HDREF_EARG;
    tr_tree t;
    int rc = tr_build(&t, len, code, A);
    if (rc != HDREF_OK) {
        free(t.nodes);
        return rc;
    }
    uint64_t pos = 0;
    for (uint64_t i = 0; i < n; ++i) {
        int64_t s = tr_step(&t, words, &pos, B);
        if (s < 0) {
            free(t.nodes);
            return HDREF_ECORRUPT;
        }
        sym_set(out, width, i, (uint32_t)s);
    }
    free(t.nodes);
    return pos == B ? HDREF_OK : HDREF_ECORRUPT;
}

int hdref_decode(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n,
                 const uint8_t *len, const uint32_t *code, uint32_t A, uint16_t *out)
{
    return hdref_decode_w(words, n_words, B, n, len, code, A, out, 2);
}

/* Decodes the first n symbols without the end-of-stream check and returns the
 * bit position reached in *end_pos (for timing a prefix of a long stream). */
int hdref_decode_prefix(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n,
                        const uint8_t *len, const uint32_t *code, uint32_t A, uint16_t *out,
                        uint64_t *end_pos)
{
    if (len == NULL || code == NULL || A == 0 || A > 65536 || (n > 0 && (out == NULL || words == NULL)))
        return HDREF_EARG;
    if (n_words * 32 < B)
        return HDREF_EARG;
    tr_tree t;
    int rc = tr_build(&t, len, code, A);
    if (rc != HDREF_OK) {
        free(t.nodes);
        return rc;
    }
    uint64_t pos = 0;
    for (uint64_t i = 0; i < n; ++i) {
        int64_t s = tr_step(&t, words, &pos, B);
        if (s < 0) {
            free(t.nodes);
            return HDREF_ECORRUPT;
        }
        out[i] = (uint16_t)s;
    }
    if (end_pos)
        *end_pos = pos;
    free(t.nodes);
    return HDREF_OK;
}

/* Decodes n symbols starting at stream bit `start`, which must be a codeword
 * start, without the end-of-stream check; the end position goes to *end_pos.
 * Ranges of chunks are independent from their first subsequence's gap entry
 * (start = k*S + gap[k]) and chunk counts (n), so a CPU baseline can run one
 * call per range on every host core (Sec. III-C: the gap array lets each
 * thread begin at a known codeword boundary). */
int hdref_decode_from_w(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t start, uint64_t n,
                        const uint8_t *len, const uint32_t *code, uint32_t A, void *out, uint32_t width,
                        uint64_t *end_pos)
{
    if (len == NULL || code == NULL || !width_fits(width, A) || (n > 0 && (out == NULL || words == NULL)))
        return HDREF_EARG;
    if (n_words * 32 < B || start > B)
        return HDREF_EARG;
    tr_tree t;
    int rc = tr_build(&t, len, code, A);
    if (rc != HDREF_OK) {
        free(t.nodes);
        return rc;
    }
    uint64_t pos = start;
    for (uint64_t i = 0; i < n; ++i) {
        int64_t s = tr_step(&t, words, &pos, B);
        if (s < 0) {
            free(t.nodes);
            return HDREF_ECORRUPT;
        }
        sym_set(out, width, i, (uint32_t)s);
    }
    if (end_pos)
        *end_pos = pos;
    free(t.nodes);
    return HDREF_OK;
}

int hdref_decode_from(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t start, uint64_t n,
                      const uint8_t *len, const uint32_t *code, uint32_t A, uint16_t *out,
                      uint64_t *end_pos)
{
    return hdref_decode_from_w(words, n_words, B, start, n, len, code, A, out, 2, end_pos);
}

/* ------------------------------------------------------------------------ */
/* Self-synchronization reference                                            */
/* ------------------------------------------------------------------------ */

/*
 * From a sequential decode of all n codewords, marks the true codeword starts
 * (plus B).  For each subsequence k:
 *   sync_gap[k]  = p_k - k*S  (the verified synchronization point);
 *   counts[k]    = number of codeword starts in [k*S, (k+1)*S);
 *   sync_bits[k] = how many bits a decoder started at the raw boundary k*S
 *                  consumes before its position is a true codeword start
 *                  (0 when k*S itself is one), or UINT32_MAX when it never
 *                  lands on one before the end of the stream.
 * Any output pointer may be NULL.
 */
int hdref_selfsync(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n,
                   const uint8_t *len, const uint32_t *code, uint32_t A, uint32_t S,
                   uint8_t *sync_gap, uint32_t *counts, uint32_t *sync_bits)
{
    if (len == NULL || code == NULL || A == 0 || A > HDREF_MAX_ALPHABET || S == 0)
        return HDREF_EARG;
    if (n_words * 32 < B || (B > 0 && words == NULL))
        return HDREF_EARG;
    tr_tree t;
    int rc = tr_build(&t, len, code, A);
    if (rc != HDREF_OK) {
        free(t.nodes);
        return rc;
    }
    uint64_t K = (B + S - 1) / S;
    uint8_t *is_start = (uint8_t *)calloc(B / 8 + 1, 1);     /* bit set per true start */
    if (!is_start) {
        free(t.nodes);
        return HDREF_ENOMEM;
    }
#define MARK(p) (is_start[(p) >> 3] |= (uint8_t)(1u << ((p) & 7)))
#define MARKED(p) ((is_start[(p) >> 3] >> ((p) & 7)) & 1u)
    uint64_t pos = 0;
    for (uint64_t i = 0; i < n; ++i) {
        MARK(pos);
        if (tr_step(&t, words, &pos, B) < 0) {
            free(t.nodes);
            free(is_start);
            return HDREF_ECORRUPT;
        }
    }
    if (pos != B) {
        free(t.nodes);
        free(is_start);
        return HDREF_ECORRUPT;
    }
    MARK(B);

    for (uint64_t k = 0; k < K; ++k) {
        uint64_t lo = k * S, hi = (k + 1) * S < B ? (k + 1) * S : B;
        if (sync_gap) {
            uint64_t p = lo;
            while (!MARKED(p))
                ++p;
            sync_gap[k] = (uint8_t)(p - lo);
        }
        if (counts) {
            uint32_t c = 0;
            for (uint64_t p = lo; p < hi; ++p)
                c += MARKED(p);
            counts[k] = c;
        }
        if (sync_bits) {
            uint64_t p = lo;
            uint32_t res = UINT32_MAX;
            for (;;) {
                if (MARKED(p)) {
                    res = (uint32_t)(p - lo);
                    break;
                }
                if (tr_step(&t, words, &p, B) < 0)
                    break;
            }
            sync_bits[k] = res;
        }
    }
#undef MARK
#undef MARKED
    free(t.nodes);
    free(is_start);
    return HDREF_OK;
}

/* Backward gap of Fig. 1: for each boundary k*S, (start of the codeword that
 * contains bit k*S) - k*S, which is <= 0.  Also the per-subsequence counts
 * under the matching ownership rule (a codeword belongs to the subsequence
 * holding its LAST bit). */
int hdref_gap_backward(const uint32_t *words, uint64_t n_words, uint64_t B, uint64_t n,
                       const uint8_t *len, const uint32_t *code, uint32_t A, uint32_t S,
                       int32_t *gapb, uint32_t *counts_b)
{
    if (len == NULL || code == NULL || A == 0 || S == 0 || n_words * 32 < B)
        return HDREF_EARG;
    tr_tree t;
    int rc = tr_build(&t, len, code, A);
    if (rc != HDREF_OK) {
        free(t.nodes);
        return rc;
    }
    uint64_t K = (B + S - 1) / S;
    for (uint64_t k = 0; k < K; ++k) {
        if (gapb)
            gapb[k] = 0;
        if (counts_b)
            counts_b[k] = 0;
    }
    uint64_t pos = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t st = pos;
        if (tr_step(&t, words, &pos, B) < 0) {
            free(t.nodes);
            return HDREF_ECORRUPT;
        }
        uint64_t last = pos - 1;
        if (counts_b)
            counts_b[last / S] += 1;
        if (gapb)
            for (uint64_t k = (st + S - 1) / S; k * S <= last && k < K; ++k)
                gapb[k] = (int32_t)((int64_t)st - (int64_t)(k * S));
    }
    free(t.nodes);
    return pos == B ? HDREF_OK : HDREF_ECORRUPT;
}
